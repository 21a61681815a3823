/*
 * tb_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for the oct-tree that the leaf-first
 * construction of Tokuue & Ishiyama (2023) produces.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library; the
 * product path never calls it.  It shares no code, header or table with the
 * HIP implementation.
 *
 * What it computes, step by step, and where each step comes from:
 *
 *   1. quantise   -- each coordinate becomes a 21-bit integer inside a root cube
 *                    whose side is a power of two (Sec. 2.2, hashed oct-tree).
 *   2. key        -- the three integers are bit-interleaved below a leading 1
 *                    bit (Sec. 2.2); x is the most significant bit of each
 *                    3-bit octant digit (a reading: the paper does not fix the
 *                    axis order).  The Peano-Hilbert variant (footnote of
 *                    Sec. 2.2) takes instead the index of the cell on the 3-D
 *                    Hilbert curve of Skilling's transpose method (J. Skilling,
 *                    "Programming the Hilbert curve", AIP Conf. Proc. 707, 381,
 *                    2004), in the same layout: a cell's key is still the upper
 *                    3d + 1 bits of its particles' keys, but a child's 3-bit digit
 *                    is its place along the curve rather than its octant.
 *   3. insertion  -- the classic Barnes-Hut top-down build (Sec. 2.1): particles
 *                    are inserted one at a time from the root; a cell that holds
 *                    more than n_leaf particles is halved along every axis and
 *                    its particles are handed to the non-empty octants.  Cells at
 *                    depth 21 (the key resolution) are never split.
 *   4. perm       -- stable order of particle indices by key, ties broken by the
 *                    original index (Sec. 2.3, step ii: sort key/index pairs).
 *                    It is cross-checked against the depth-first order of the
 *                    top-down tree.
 *   5. canonical  -- cells listed by (depth, key) ascending; each cell records
 *                    its key (Sec. 2.2: root = 1, child = parent<<3 | octant),
 *                    depth, the first sorted position and count of its particles,
 *                    and its first child and number of children.
 *   6. moments    -- for every cell, straight from its own particle set (never
 *                    from its children): mass, centre of mass and the traceless
 *                    quadrupole about the centre of mass (Sec. 2.3.2: cell
 *                    properties; footnote: higher multipoles likewise, centre of
 *                    the cell from its depth and key).  Sums are FP64 with
 *                    Neumaier compensation; the quadrupole is a second pass
 *                    about the finished centre of mass.
 *
 * Frames.  A particle's box-frame position is u = fl64(x - lo), the same value
 * that quantisation scales by 2^21/side.  A cell's geometric centre in that
 * frame is off = (ijk + 1/2) * side * 2^-depth, which is exact.  The stored
 * centre of mass is com_rel = sum m*(u - off) / M, i.e. relative to the cell
 * centre, and the quadrupole is Q_ab = sum m (3 r_a r_b - |r|^2 delta_ab) with
 * r = (u - off) - com_rel.
 *
 * Build with -O2 -ffp-contract=off and no fast-math, so every FP64 operation is
 * a single IEEE round-to-nearest step.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define TBO_OK 0
#define TBO_ERR_ARG (-1)
#define TBO_ERR_BOX (-2)
#define TBO_ERR_NONFINITE (-5)
#define TBO_ERR_MASS (-6)
#define TBO_ERR_NOMEM (-7)
#define TBO_ERR_INTERNAL (-8)

#define TBO_MAX_DEPTH 21
#define TBO_QMAX 2097151u /* 2^21 - 1 */

/* ---------------------------------------------------------------------- */
/* Step 1-2: quantisation and key (Sec. 2.2)                               */
/* ---------------------------------------------------------------------- */

static int side_is_pow2(double side) {
  int e;
  if (!(side > 0.0) || !isfinite(side)) return 0;
  return frexp(side, &e) == 0.5;
}

/* One coordinate -> 21-bit integer: floor((x - lo) * 2^21 / side), clamped
 * into [0, 2^21 - 1].  2^21/side is a power of two, so the product is exact and
 * the only rounding is the subtraction. */
static uint32_t quantise1(float x, double lo, double scale) {
  double u = (double)x - lo;
  double t = u * scale;
  if (!(t >= 0.0)) return 0u; /* also catches NaN */
  if (t >= 2097152.0) return TBO_QMAX;
  return (uint32_t)floor(t);
}

/* Interleave one bit at a time: for bit b (20 down to 0) append x_b, y_b, z_b
 * after a leading 1. */
static uint64_t interleave_key(uint32_t qx, uint32_t qy, uint32_t qz) {
  uint64_t k = 1u;
  int b;
  for (b = TBO_MAX_DEPTH - 1; b >= 0; --b) {
    k = (k << 1) | ((qx >> b) & 1u);
    k = (k << 1) | ((qy >> b) & 1u);
    k = (k << 1) | ((qz >> b) & 1u);
  }
  return k;
}

/* Peano-Hilbert index of cell (x, y, z) on the curve of `bits` levels
 * (Skilling's method).  First the coordinates become the curve's "transposed"
 * index: from the top level down, a coordinate whose bit at this level is set
 * inverts the lower bits of x, and one whose bit is clear exchanges its lower
 * bits with those of x; then a Gray-code decode along x, y, z.  The index's
 * digit at each level is (x, y, z) of the transposed form at that level, x the
 * most significant.  Bits 3*bits-1 .. 0 of the result; no leading 1. */
static uint64_t hilbert_encode(uint32_t x, uint32_t y, uint32_t z, int bits) {
  uint32_t X[3], Q, P, t;
  uint64_t h = 0;
  int i, b;
  X[0] = x;
  X[1] = y;
  X[2] = z;
  if (bits <= 0) return 0;
  for (Q = 1u << (bits - 1); Q > 1u; Q >>= 1) {
    P = Q - 1u;
    for (i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  t = 0;
  for (Q = 1u << (bits - 1); Q > 1u; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1u;
  for (i = 0; i < 3; ++i) X[i] ^= t;
  for (b = bits - 1; b >= 0; --b)
    for (i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
  return h;
}

/* Inverse of hilbert_encode: cell coordinates of index h on the curve of
 * `bits` levels. */
static void hilbert_decode(uint64_t h, int bits, uint32_t q[3]) {
  uint32_t X[3] = {0u, 0u, 0u}, N, Q, P, t;
  int i, b;
  for (b = bits - 1; b >= 0; --b)
    for (i = 0; i < 3; ++i) X[i] |= (uint32_t)((h >> (3 * b + 2 - i)) & 1u) << b;
  if (bits > 0) {
    N = 2u << (bits - 1);
    t = X[2] >> 1;
    X[2] ^= X[1];
    X[1] ^= X[0];
    X[0] ^= t;
    for (Q = 2u; Q != N; Q <<= 1) {
      P = Q - 1u;
      for (i = 2; i >= 0; --i) {
        if (X[i] & Q) {
          X[0] ^= P;
        } else {
          t = (X[0] ^ X[i]) & P;
          X[0] ^= t;
          X[i] ^= t;
        }
      }
    }
  }
  q[0] = X[0];
  q[1] = X[1];
  q[2] = X[2];
}

void tbo_hilbert_encode(const uint32_t *q /* [n][3] */, int64_t n, int bits, uint64_t *h) {
  int64_t i;
  for (i = 0; i < n; ++i) h[i] = hilbert_encode(q[3 * i], q[3 * i + 1], q[3 * i + 2], bits);
}

void tbo_hilbert_decode(const uint64_t *h, int64_t n, int bits, uint32_t *q /* [n][3] */) {
  int64_t i;
  for (i = 0; i < n; ++i) hilbert_decode(h[i], bits, &q[3 * i]);
}

/* curve 0: Morton keys; 1: Peano-Hilbert keys, each below a leading 1. */
int tbo_keys_curve(const float *pos, int64_t n, const double lo[3], double side, int curve,
                   uint32_t *q_out /* [n][3] or NULL */, uint64_t *key_out /* [n] */) {
  double scale;
  int64_t i;
  if (n < 0 || (n > 0 && (!pos || !key_out)) || !lo || curve < 0 || curve > 1)
    return TBO_ERR_ARG;
  if (!side_is_pow2(side) || !isfinite(lo[0]) || !isfinite(lo[1]) || !isfinite(lo[2]))
    return TBO_ERR_BOX;
  scale = ldexp(1.0, 21) / side;
  for (i = 0; i < n; ++i) {
    uint32_t q0 = quantise1(pos[3 * i + 0], lo[0], scale);
    uint32_t q1 = quantise1(pos[3 * i + 1], lo[1], scale);
    uint32_t q2 = quantise1(pos[3 * i + 2], lo[2], scale);
    if (q_out) {
      q_out[3 * i + 0] = q0;
      q_out[3 * i + 1] = q1;
      q_out[3 * i + 2] = q2;
    }
    key_out[i] = curve ? ((uint64_t)1 << 63) | hilbert_encode(q0, q1, q2, TBO_MAX_DEPTH)
                       : interleave_key(q0, q1, q2);
  }
  return TBO_OK;
}

int tbo_keys(const float *pos, int64_t n, const double lo[3], double side,
             uint32_t *q_out /* [n][3] or NULL */, uint64_t *key_out /* [n] */) {
  return tbo_keys_curve(pos, n, lo, side, 0, q_out, key_out);
}

/* ---------------------------------------------------------------------- */
/* Step 3: top-down insertion (Sec. 2.1)                                   */
/* ---------------------------------------------------------------------- */

typedef struct {
  int level;
  uint64_t key;
  int child[8]; /* node index or -1 */
  int is_leaf;
  int32_t *mem; /* particle indices held by a leaf */
  int64_t cnt, cap;
  /* filled during canonicalisation */
  int64_t canon;
  int64_t first, count;
} tbo_node;

typedef struct {
  tbo_node *v;
  int64_t n, cap;
  const uint32_t *q;
  const uint64_t *keys; /* particle keys: a child's key is their prefix */
  int32_t n_leaf;
  int failed;
} tbo_tree;

static int64_t new_node(tbo_tree *t, int level, uint64_t key) {
  tbo_node *nd;
  int c;
  if (t->n == t->cap) {
    int64_t nc = t->cap ? 2 * t->cap : 64;
    tbo_node *nv = (tbo_node *)realloc(t->v, (size_t)nc * sizeof(tbo_node));
    if (!nv) {
      t->failed = 1;
      return -1;
    }
    t->v = nv;
    t->cap = nc;
  }
  nd = &t->v[t->n];
  memset(nd, 0, sizeof(*nd));
  nd->level = level;
  nd->key = key;
  for (c = 0; c < 8; ++c) nd->child[c] = -1;
  nd->is_leaf = 1;
  return t->n++;
}

static int push_member(tbo_tree *t, int64_t node, int32_t p) {
  tbo_node *nd = &t->v[node];
  if (nd->cnt == nd->cap) {
    int64_t nc = nd->cap ? 2 * nd->cap : 4;
    int32_t *nm = (int32_t *)realloc(nd->mem, (size_t)nc * sizeof(int32_t));
    if (!nm) {
      t->failed = 1;
      return -1;
    }
    nd->mem = nm;
    nd->cap = nc;
  }
  nd->mem[nd->cnt++] = p;
  return 0;
}

/* Octant of particle p below a cell at depth `level`: the (20-level)-th bit of
 * each coordinate, x most significant. */
static int octant_of(const tbo_tree *t, int32_t p, int level) {
  int b = TBO_MAX_DEPTH - 1 - level;
  const uint32_t *q = &t->q[3 * (int64_t)p];
  return (int)((((q[0] >> b) & 1u) << 2) | (((q[1] >> b) & 1u) << 1) | ((q[2] >> b) & 1u));
}

/* The child of `node` in octant `oct`, created for particle p if missing.  Its
 * key is the prefix of p's key (for Morton keys, the parent's key followed by
 * the octant). */
static int64_t child_for(tbo_tree *t, int64_t node, int oct, int32_t p) {
  int64_t c = t->v[node].child[oct];
  if (c < 0) {
    int lvl = t->v[node].level + 1;
    uint64_t key = t->keys[p] >> (3 * (TBO_MAX_DEPTH - lvl));
    c = new_node(t, lvl, key); /* may move t->v */
    if (c < 0) return -1;
    t->v[node].child[oct] = (int)c;
  }
  return c;
}

/* Halve a leaf that holds more than n_leaf particles; recurse into children
 * that still hold too many. */
static void split(tbo_tree *t, int64_t node) {
  int32_t *mem;
  int64_t cnt, k;
  int oct;
  if (t->failed) return;
  if (t->v[node].cnt <= t->n_leaf || t->v[node].level >= TBO_MAX_DEPTH) return;
  mem = t->v[node].mem;
  cnt = t->v[node].cnt;
  t->v[node].mem = NULL;
  t->v[node].cnt = t->v[node].cap = 0;
  t->v[node].is_leaf = 0;
  for (k = 0; k < cnt && !t->failed; ++k) {
    int32_t p = mem[k];
    int64_t c = child_for(t, node, octant_of(t, p, t->v[node].level), p);
    if (c < 0) break;
    push_member(t, c, p);
  }
  free(mem);
  for (oct = 0; oct < 8 && !t->failed; ++oct) {
    int64_t c = t->v[node].child[oct];
    if (c >= 0) split(t, c);
  }
}

static void insert(tbo_tree *t, int32_t p) {
  int64_t node = 0;
  while (!t->v[node].is_leaf) {
    node = child_for(t, node, octant_of(t, p, t->v[node].level), p);
    if (node < 0) return;
  }
  if (push_member(t, node, p) < 0) return;
  split(t, node);
}

/* ---------------------------------------------------------------------- */
/* Step 4: perm by a library sort; DFS order cross-check                   */
/* ---------------------------------------------------------------------- */

typedef struct {
  uint64_t key;
  int32_t idx;
} tbo_pair;

static int cmp_pair(const void *a, const void *b) {
  const tbo_pair *x = (const tbo_pair *)a, *y = (const tbo_pair *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

static const uint64_t *g_keys_for_cmp; /* qsort has no context argument */
static int cmp_idx_by_key(const void *a, const void *b) {
  int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
  uint64_t ki = g_keys_for_cmp[i], kj = g_keys_for_cmp[j];
  if (ki != kj) return ki < kj ? -1 : 1;
  return (i > j) - (i < j);
}

/* The children of a node in key order (for Morton keys, octant order); returns
 * how many. */
static int children_by_key(const tbo_tree *t, int64_t node, int64_t out[8]) {
  int n = 0, oct, k;
  for (oct = 0; oct < 8; ++oct) {
    int64_t c = t->v[node].child[oct];
    if (c < 0) continue;
    for (k = n; k > 0 && t->v[out[k - 1]].key > t->v[c].key; --k) out[k] = out[k - 1];
    out[k] = c;
    ++n;
  }
  return n;
}

/* Depth-first walk: children in key order; a leaf's particles by (key, index). */
static void dfs_emit(tbo_tree *t, int64_t node, const uint64_t *keys, int32_t *out, int64_t *w) {
  tbo_node *nd = &t->v[node];
  int64_t ch[8];
  int k, nch;
  if (nd->is_leaf) {
    int64_t j;
    g_keys_for_cmp = keys;
    qsort(nd->mem, (size_t)nd->cnt, sizeof(int32_t), cmp_idx_by_key);
    for (j = 0; j < nd->cnt; ++j) out[(*w)++] = nd->mem[j];
    return;
  }
  nch = children_by_key(t, node, ch);
  for (k = 0; k < nch; ++k) dfs_emit(t, ch[k], keys, out, w);
}

/* ---------------------------------------------------------------------- */
/* Step 5: canonical (depth, key) order                                    */
/* ---------------------------------------------------------------------- */

static const tbo_node *g_nodes_for_cmp;
static int cmp_node(const void *a, const void *b) {
  const tbo_node *x = &g_nodes_for_cmp[*(const int64_t *)a];
  const tbo_node *y = &g_nodes_for_cmp[*(const int64_t *)b];
  if (x->level != y->level) return x->level < y->level ? -1 : 1;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Step 6: moments straight from each cell's particles                     */
/* ---------------------------------------------------------------------- */

/* Neumaier's compensated summation. */
typedef struct {
  double s, c;
} tbo_sum;
static void nsum_add(tbo_sum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static double nsum_val(const tbo_sum *a) { return a->s + a->c; }

/* Cell centre in the box frame: (ijk + 1/2) * side * 2^-level per axis, with
 * ijk read back out of the cell key (curve 1: decoded from the Hilbert index
 * below the leading 1). */
static void cell_offset(uint64_t key, int level, double side, int curve, double off[3]) {
  uint32_t ijk[3] = {0u, 0u, 0u};
  int l;
  double h = ldexp(side, -level);
  if (curve) {
    hilbert_decode(key & (((uint64_t)1 << (3 * level)) - 1u), level, ijk);
  } else {
    for (l = 0; l < level; ++l) {
      int sh = 3 * (level - 1 - l);
      ijk[0] = (ijk[0] << 1) | (uint32_t)((key >> (sh + 2)) & 1u);
      ijk[1] = (ijk[1] << 1) | (uint32_t)((key >> (sh + 1)) & 1u);
      ijk[2] = (ijk[2] << 1) | (uint32_t)((key >> sh) & 1u);
    }
  }
  off[0] = ((double)ijk[0] + 0.5) * h;
  off[1] = ((double)ijk[1] + 0.5) * h;
  off[2] = ((double)ijk[2] + 0.5) * h;
}

static void cell_moments(const float *pos, const float *mass, const double lo[3], double side,
                         const int32_t *perm, int64_t first, int64_t count, uint64_t key,
                         int level, int curve, double com_out[4], double quad_out[6]) {
  double off[3], M, c[3];
  tbo_sum sm = {0, 0}, s1[3] = {{0, 0}, {0, 0}, {0, 0}};
  tbo_sum s2[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  int64_t k;
  int a;
  cell_offset(key, level, side, curve, off);
  /* pass 1: mass and centre of mass */
  for (k = first; k < first + count; ++k) {
    int32_t p = perm[k];
    double m = (double)mass[p];
    nsum_add(&sm, m);
    for (a = 0; a < 3; ++a) {
      double r = ((double)pos[3 * (int64_t)p + a] - lo[a]) - off[a];
      nsum_add(&s1[a], m * r);
    }
  }
  M = nsum_val(&sm);
  for (a = 0; a < 3; ++a) c[a] = nsum_val(&s1[a]) / M;
  /* pass 2: traceless quadrupole about the centre of mass */
  for (k = first; k < first + count; ++k) {
    int32_t p = perm[k];
    double m = (double)mass[p], r[3], r2;
    for (a = 0; a < 3; ++a) r[a] = (((double)pos[3 * (int64_t)p + a] - lo[a]) - off[a]) - c[a];
    r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    nsum_add(&s2[0], m * (3.0 * r[0] * r[0] - r2));
    nsum_add(&s2[1], m * (3.0 * r[0] * r[1]));
    nsum_add(&s2[2], m * (3.0 * r[0] * r[2]));
    nsum_add(&s2[3], m * (3.0 * r[1] * r[1] - r2));
    nsum_add(&s2[4], m * (3.0 * r[1] * r[2]));
    nsum_add(&s2[5], m * (3.0 * r[2] * r[2] - r2));
  }
  com_out[0] = c[0];
  com_out[1] = c[1];
  com_out[2] = c[2];
  com_out[3] = M;
  for (a = 0; a < 6; ++a) quad_out[a] = nsum_val(&s2[a]);
}

/* ---------------------------------------------------------------------- */
/* Public entry points                                                     */
/* ---------------------------------------------------------------------- */

/* Wall-clock seconds (monotonic), for the optional per-stage timings. */
static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Upper bound on the number of cells: at most N leaves, and at each of the
 * depths 0..20 at most floor(N/(n_leaf+1)) split cells (they are disjoint and
 * each holds more than n_leaf particles). */
int64_t tbo_max_cells(int64_t n, int32_t n_leaf) {
  if (n <= 0 || n_leaf < 1) return 0;
  return n + (int64_t)TBO_MAX_DEPTH * (n / ((int64_t)n_leaf + 1));
}

/*
 * Full reference build.  All pointers are host memory, caller-owned:
 *   pos [n][3], mass [n]                       inputs
 *   perm [n]                                   stable key order
 *   dfs_perm [n] (may be NULL)                 depth-first order of the top-down tree
 *   cell_* [tbo_max_cells]                     canonical (depth, key) order
 *   child_ptr [cells][2]                       {first child, #children}, leaf {-1, 0}
 *   com [cells][4], quad [cells][6]            moments (NULL to skip them)
 *   level_offset [23]                          first cell of each depth, [22] = n_cells
 * Returns 0 or a negative error code; *n_cells receives the number of cells.
 * stage_s [5] (may be NULL) receives the seconds spent in steps 1-2 (keys),
 * 3 (insertion), 4 (perm and its DFS cross-check), 5 (canonical order, ranges,
 * child links) and 6 (moments).
 */
int tbo_build_curve(const float *pos, const float *mass, int64_t n, int32_t n_leaf,
                    const double lo[3], double side, int curve, int32_t *perm, int32_t *dfs_perm,
                    uint64_t *cell_key, uint8_t *cell_level, int32_t *cell_first,
                    int32_t *cell_count, int32_t *child_ptr, double *com, double *quad,
                    int64_t *level_offset, int64_t *n_cells, double *stage_s) {
  tbo_tree t;
  uint32_t *q = NULL;
  uint64_t *keys = NULL;
  tbo_pair *pairs = NULL;
  int32_t *dfs = NULL;
  int64_t *order = NULL, *pos_of = NULL;
  int64_t i, c, nc;
  int rc = TBO_OK, lvl;
  double t0 = now_s(), t1;

  if (stage_s)
    for (lvl = 0; lvl < 5; ++lvl) stage_s[lvl] = 0.0;
  if (n < 0 || n > 2147483647LL || n_leaf < 1 || !lo || !n_cells || !level_offset || curve < 0 ||
      curve > 1)
    return TBO_ERR_ARG;
  if (n > 0 && (!pos || !mass || !perm || !cell_key || !cell_level || !cell_first ||
                !cell_count || !child_ptr))
    return TBO_ERR_ARG;
  if (!side_is_pow2(side) || !isfinite(lo[0]) || !isfinite(lo[1]) || !isfinite(lo[2]))
    return TBO_ERR_BOX;
  for (i = 0; i < 3 * n; ++i)
    if (!isfinite(pos[i])) return TBO_ERR_NONFINITE;
  for (i = 0; i < n; ++i)
    if (!(mass[i] > 0.0f) || !isfinite(mass[i])) return TBO_ERR_MASS;
  for (lvl = 0; lvl <= TBO_MAX_DEPTH + 1; ++lvl) level_offset[lvl] = 0;
  *n_cells = 0;
  if (n == 0) return TBO_OK;

  memset(&t, 0, sizeof(t));
  q = (uint32_t *)malloc((size_t)n * 3 * sizeof(uint32_t));
  keys = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  pairs = (tbo_pair *)malloc((size_t)n * sizeof(tbo_pair));
  dfs = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  pos_of = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  if (!q || !keys || !pairs || !dfs || !pos_of) {
    rc = TBO_ERR_NOMEM;
    goto done;
  }
  rc = tbo_keys_curve(pos, n, lo, side, curve, q, keys);
  if (rc) goto done;
  t1 = now_s();
  if (stage_s) stage_s[0] = t1 - t0;
  t0 = t1;

  /* step 3: top-down insertion in index order */
  t.q = q;
  t.keys = keys;
  t.n_leaf = n_leaf;
  if (new_node(&t, 0, 1u) < 0) {
    rc = TBO_ERR_NOMEM;
    goto done;
  }
  for (i = 0; i < n && !t.failed; ++i) insert(&t, (int32_t)i);
  if (t.failed) {
    rc = TBO_ERR_NOMEM;
    goto done;
  }
  t1 = now_s();
  if (stage_s) stage_s[1] = t1 - t0;
  t0 = t1;

  /* step 4: perm = stable key order; cross-check with the DFS order */
  for (i = 0; i < n; ++i) {
    pairs[i].key = keys[i];
    pairs[i].idx = (int32_t)i;
  }
  qsort(pairs, (size_t)n, sizeof(tbo_pair), cmp_pair);
  for (i = 0; i < n; ++i) {
    perm[i] = pairs[i].idx;
    pos_of[pairs[i].idx] = i;
  }
  {
    int64_t w = 0;
    dfs_emit(&t, 0, keys, dfs, &w);
    if (w != n) {
      rc = TBO_ERR_INTERNAL;
      goto done;
    }
    for (i = 0; i < n; ++i)
      if (dfs[i] != perm[i]) {
        rc = TBO_ERR_INTERNAL;
        goto done;
      }
    if (dfs_perm) memcpy(dfs_perm, dfs, (size_t)n * sizeof(int32_t));
  }
  t1 = now_s();
  if (stage_s) stage_s[2] = t1 - t0;
  t0 = t1;

  /* step 5: canonical order */
  nc = t.n;
  if (nc > tbo_max_cells(n, n_leaf)) {
    rc = TBO_ERR_INTERNAL;
    goto done;
  }
  order = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
  if (!order) {
    rc = TBO_ERR_NOMEM;
    goto done;
  }
  for (c = 0; c < nc; ++c) order[c] = c;
  g_nodes_for_cmp = t.v;
  qsort(order, (size_t)nc, sizeof(int64_t), cmp_node);
  for (c = 0; c < nc; ++c) t.v[order[c]].canon = c;

  /* particle ranges, deepest cells first so children are ready for parents */
  for (c = nc - 1; c >= 0; --c) {
    tbo_node *nd = &t.v[order[c]];
    if (nd->is_leaf) {
      int64_t lo_s = n, hi_s = -1, k;
      for (k = 0; k < nd->cnt; ++k) {
        int64_t s = pos_of[nd->mem[k]];
        if (s < lo_s) lo_s = s;
        if (s > hi_s) hi_s = s;
      }
      nd->first = lo_s;
      nd->count = nd->cnt;
      if (nd->cnt < 1 || hi_s - lo_s + 1 != nd->cnt) {
        rc = TBO_ERR_INTERNAL; /* a leaf's particles must be contiguous in key order */
        goto done;
      }
    } else {
      int64_t first = -1, end = -1, cnt = 0, chs[8];
      int k, nch = children_by_key(&t, order[c], chs);
      for (k = 0; k < nch; ++k) {
        int64_t ch = chs[k];
        if (first < 0) {
          first = t.v[ch].first;
        } else if (t.v[ch].first != end) {
          rc = TBO_ERR_INTERNAL; /* children must tile the parent's range */
          goto done;
        }
        end = t.v[ch].first + t.v[ch].count;
        cnt += t.v[ch].count;
      }
      nd->first = first;
      nd->count = cnt;
    }
  }

  for (c = 0; c < nc; ++c) {
    tbo_node *nd = &t.v[order[c]];
    int64_t chs[8];
    int nchild = children_by_key(&t, order[c], chs);
    int64_t first_child = nchild > 0 ? t.v[chs[0]].canon : -1;
    cell_key[c] = nd->key;
    cell_level[c] = (uint8_t)nd->level;
    cell_first[c] = (int32_t)nd->first;
    cell_count[c] = (int32_t)nd->count;
    child_ptr[2 * c] = nd->is_leaf ? -1 : (int32_t)first_child;
    child_ptr[2 * c + 1] = nd->is_leaf ? 0 : nchild;
  }
  for (lvl = 0; lvl <= TBO_MAX_DEPTH + 1; ++lvl) level_offset[lvl] = nc;
  for (c = nc - 1; c >= 0; --c) level_offset[cell_level[c]] = c;
  for (lvl = TBO_MAX_DEPTH; lvl >= 0; --lvl)
    if (level_offset[lvl] > level_offset[lvl + 1]) level_offset[lvl] = level_offset[lvl + 1];
  *n_cells = nc;
  t1 = now_s();
  if (stage_s) stage_s[3] = t1 - t0;
  t0 = t1;

  /* step 6: moments */
  if (com && quad) {
    for (c = 0; c < nc; ++c)
      cell_moments(pos, mass, lo, side, perm, cell_first[c], cell_count[c], cell_key[c],
                   cell_level[c], curve, &com[4 * c], &quad[6 * c]);
  }
  if (stage_s) stage_s[4] = now_s() - t0;

done:
  for (i = 0; i < t.n; ++i) free(t.v[i].mem);
  free(t.v);
  free(q);
  free(keys);
  free(pairs);
  free(dfs);
  free(pos_of);
  free(order);
  return rc;
}

int tbo_build_timed(const float *pos, const float *mass, int64_t n, int32_t n_leaf,
                    const double lo[3], double side, int32_t *perm, int32_t *dfs_perm,
                    uint64_t *cell_key, uint8_t *cell_level, int32_t *cell_first,
                    int32_t *cell_count, int32_t *child_ptr, double *com, double *quad,
                    int64_t *level_offset, int64_t *n_cells, double *stage_s) {
  return tbo_build_curve(pos, mass, n, n_leaf, lo, side, 0, perm, dfs_perm, cell_key, cell_level,
                         cell_first, cell_count, child_ptr, com, quad, level_offset, n_cells,
                         stage_s);
}

int tbo_build(const float *pos, const float *mass, int64_t n, int32_t n_leaf, const double lo[3],
              double side, int32_t *perm, int32_t *dfs_perm, uint64_t *cell_key,
              uint8_t *cell_level, int32_t *cell_first, int32_t *cell_count, int32_t *child_ptr,
              double *com, double *quad, int64_t *level_offset, int64_t *n_cells) {
  return tbo_build_timed(pos, mass, n, n_leaf, lo, side, perm, dfs_perm, cell_key, cell_level,
                         cell_first, cell_count, child_ptr, com, quad, level_offset, n_cells,
                         NULL);
}

/* Moments of one arbitrary particle range [first, first+count) of `perm`, in the
 * frame of the cell (key, level).  Lets tests sample single cells of very large
 * trees without rebuilding the whole tree on the CPU. */
int tbo_cell_moments(const float *pos, const float *mass, const double lo[3], double side,
                     const int32_t *perm, int64_t first, int64_t count, uint64_t key, int level,
                     double com_out[4], double quad_out[6]) {
  if (!pos || !mass || !lo || !perm || !com_out || !quad_out || count < 1 || first < 0 ||
      level < 0 || level > TBO_MAX_DEPTH)
    return TBO_ERR_ARG;
  if (!side_is_pow2(side)) return TBO_ERR_BOX;
  cell_moments(pos, mass, lo, side, perm, first, count, key, level, 0, com_out, quad_out);
  return TBO_OK;
}

/* Root box for a point set: lo = per-axis minimum, side = the smallest power of
 * two strictly larger than the largest extent (1 if every extent is 0). */
int tbo_auto_box(const float *pos, int64_t n, double lo[3], double *side) {
  double mn[3], mx[3], ext = 0.0, s;
  int64_t i;
  int a;
  if (n < 1 || !pos || !lo || !side) return TBO_ERR_ARG;
  for (a = 0; a < 3; ++a) mn[a] = mx[a] = (double)pos[a];
  for (i = 0; i < n; ++i)
    for (a = 0; a < 3; ++a) {
      double v = (double)pos[3 * i + a];
      if (!isfinite(v)) return TBO_ERR_NONFINITE;
      if (v < mn[a]) mn[a] = v;
      if (v > mx[a]) mx[a] = v;
    }
  for (a = 0; a < 3; ++a) {
    lo[a] = mn[a];
    if (mx[a] - mn[a] > ext) ext = mx[a] - mn[a];
  }
  if (ext == 0.0) {
    *side = 1.0;
    return TBO_OK;
  }
  s = 1.0;
  while (s <= ext) s *= 2.0;
  while (s * 0.5 > ext) s *= 0.5;
  *side = s;
  return TBO_OK;
}
