/*
 * tb_leaffirst.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The leaf-first construction of Tokuue & Ishiyama (2023), Sec. 2.3, on one
 * CPU thread, as the paper describes it.  It is a second CPU reference: the
 * tests pin it against the top-down oracle (tb_oracle.c), and the benchmark
 * times it beside the oracle as the paper's own method on a CPU core.  Only
 * the test suite and the benchmark's CPU-baseline leg may load it; it shares
 * no code with the HIP implementation.
 *
 * Steps, in the paper's order (Sec. 2.3, steps i-iv):
 *   (i)   particle keys: the oracle's FP64 quantisation and bit interleave
 *         (tbo_keys, Sec. 2.2);
 *   (ii)  sort of (key, index) pairs, equal keys by index;
 *   (iii) reorder of positions and masses into key order;
 *   (iv)  cells, leaves first (Sec. 2.3.1, Algorithm 1): the first particle k of
 *         a leaf fixes the leaf depth D_k as the larger of minDepth(k-1, k) and
 *         minDepth(k, k + n_leaf) (a missing neighbour contributes 0; depth
 *         capped at the 21-bit key resolution), and the leaf takes every
 *         following particle whose upper 3 D_k + 1 key bits equal its own.  Each
 *         leaf's moments are computed when it is created.
 *   (v)   then the parents, one depth at a time from the deepest (Sec. 2.3.2,
 *         Algorithm 2): the leaves and the inner cells of depth d are two lists
 *         sorted by key; they are consumed together in key order, and a cell
 *         whose key >> 3 differs from the last parent's key opens a new parent
 *         at depth d - 1 and closes the previous one, whose moments are then
 *         combined from its children (Sec. 2.3.2, its footnotes).  The parent
 *         still open when the lists run out is closed after the loop.
 *
 * Moments: a leaf sums m, m r and m r r over its particles with r relative to
 * its geometric centre (plain FP64 sums), then takes the centre of mass and the
 * traceless quadrupole about it.  A parent combines its children in its own
 * frame: child centres sit at +-l/4 per axis from the parent centre (l the
 * parent side, the sign from the child's octant bit), M = sum M_c,
 * com = sum M_c (com_c + s_c) / M, Q = sum [Q_c + M_c (3 d d - |d|^2 I)] with
 * d = com_c + s_c - com.  The layout of the output is that of tbo_build.
 *
 * Built, like the oracle, with -ffp-contract=off and no fast-math.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define TBL_OK 0
#define TBL_ERR_ARG (-1)
#define TBL_ERR_BOX (-2)
#define TBL_ERR_NONFINITE (-5)
#define TBL_ERR_MASS (-6)
#define TBL_ERR_NOMEM (-7)
#define TBL_ERR_INTERNAL (-8)

#define TBL_MAX_DEPTH 21
#define TBL_LEVELS (TBL_MAX_DEPTH + 1)

/* The oracle's key function (tb_oracle.c). */
int tbo_keys(const float *pos, int64_t n, const double lo[3], double side, uint32_t *q_out,
             uint64_t *key_out);

typedef struct {
  uint64_t key;
  int64_t first, count;
  int64_t child; /* index of the first child in the next depth's list, -1 for a leaf */
  int nchild;
  double com[4], quad[6];
} tbl_cell;

typedef struct {
  tbl_cell *v;
  int64_t n, cap;
} tbl_list;

static tbl_cell *list_push(tbl_list *l) {
  if (l->n == l->cap) {
    int64_t nc = l->cap ? 2 * l->cap : 256;
    tbl_cell *nv = (tbl_cell *)realloc(l->v, (size_t)nc * sizeof(tbl_cell));
    if (!nv) return NULL;
    l->v = nv;
    l->cap = nc;
  }
  memset(&l->v[l->n], 0, sizeof(tbl_cell));
  return &l->v[l->n++];
}

static double seconds(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

typedef struct {
  uint64_t key;
  int32_t idx;
} tbl_pair;

static int cmp_key_idx(const void *a, const void *b) {
  const tbl_pair *x = (const tbl_pair *)a, *y = (const tbl_pair *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

/* minDepth of two particle keys: leading zeros of the XOR over three, rounded
 * up; identical keys have no distinguishing bit (64 zeros -> 22). */
static int min_depth(uint64_t a, uint64_t b) {
  uint64_t x = a ^ b;
  int z = x ? __builtin_clzll(x) : 64;
  return (z + 2) / 3;
}

/* The depth-d cell key of a particle key: its upper 3d + 1 bits. */
static uint64_t cell_key_of(uint64_t key, int d) { return key >> (63 - 3 * d); }

/* Geometric centre of a cell in the box frame, from its depth and key. */
static void centre_of(uint64_t key, int d, double side, double c[3]) {
  uint32_t ijk[3] = {0u, 0u, 0u};
  int l, a;
  double h = ldexp(side, -d);
  for (l = d - 1; l >= 0; --l) {
    uint32_t oct = (uint32_t)((key >> (3 * l)) & 7u);
    ijk[0] = (ijk[0] << 1) | ((oct >> 2) & 1u);
    ijk[1] = (ijk[1] << 1) | ((oct >> 1) & 1u);
    ijk[2] = (ijk[2] << 1) | (oct & 1u);
  }
  for (a = 0; a < 3; ++a) c[a] = ((double)ijk[a] + 0.5) * h;
}

/* Leaf moments from its particles (sorted arrays spos/smass, range [f, f+cnt)). */
static void leaf_moments(tbl_cell *c, int d, const float *spos, const float *smass,
                         const double lo[3], double side) {
  double off[3], M = 0.0, s1[3] = {0.0, 0.0, 0.0}, com[3], q[6] = {0, 0, 0, 0, 0, 0};
  int64_t k;
  int a;
  centre_of(c->key, d, side, off);
  for (k = c->first; k < c->first + c->count; ++k) {
    double m = (double)smass[k];
    M += m;
    for (a = 0; a < 3; ++a) s1[a] += m * (((double)spos[3 * k + a] - lo[a]) - off[a]);
  }
  for (a = 0; a < 3; ++a) com[a] = s1[a] / M;
  for (k = c->first; k < c->first + c->count; ++k) {
    double m = (double)smass[k], r[3], r2;
    for (a = 0; a < 3; ++a) r[a] = (((double)spos[3 * k + a] - lo[a]) - off[a]) - com[a];
    r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    q[0] += m * (3.0 * r[0] * r[0] - r2);
    q[1] += m * (3.0 * r[0] * r[1]);
    q[2] += m * (3.0 * r[0] * r[2]);
    q[3] += m * (3.0 * r[1] * r[1] - r2);
    q[4] += m * (3.0 * r[1] * r[2]);
    q[5] += m * (3.0 * r[2] * r[2] - r2);
  }
  for (a = 0; a < 3; ++a) c->com[a] = com[a];
  c->com[3] = M;
  for (a = 0; a < 6; ++a) c->quad[a] = q[a];
}

/* A closed parent at depth d - 1 combines its children kids[0 .. n) (depth d). */
static void parent_moments(tbl_cell *p, int d, const tbl_cell *kids, double side) {
  const double quarter = ldexp(side, -(d + 1)); /* l_parent / 4 */
  double M = 0.0, s[3] = {0.0, 0.0, 0.0}, com[3], q[6] = {0, 0, 0, 0, 0, 0};
  int k, a;
  for (k = 0; k < p->nchild; ++k) {
    const tbl_cell *c = &kids[k];
    uint32_t oct = (uint32_t)(c->key & 7u);
    double u[3];
    u[0] = c->com[0] + ((oct & 4u) ? quarter : -quarter);
    u[1] = c->com[1] + ((oct & 2u) ? quarter : -quarter);
    u[2] = c->com[2] + ((oct & 1u) ? quarter : -quarter);
    M += c->com[3];
    for (a = 0; a < 3; ++a) s[a] += c->com[3] * u[a];
  }
  for (a = 0; a < 3; ++a) com[a] = s[a] / M;
  for (k = 0; k < p->nchild; ++k) {
    const tbl_cell *c = &kids[k];
    uint32_t oct = (uint32_t)(c->key & 7u);
    double dv[3], dd, m = c->com[3];
    dv[0] = c->com[0] + ((oct & 4u) ? quarter : -quarter) - com[0];
    dv[1] = c->com[1] + ((oct & 2u) ? quarter : -quarter) - com[1];
    dv[2] = c->com[2] + ((oct & 1u) ? quarter : -quarter) - com[2];
    dd = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    q[0] += c->quad[0] + m * (3.0 * dv[0] * dv[0] - dd);
    q[1] += c->quad[1] + m * (3.0 * dv[0] * dv[1]);
    q[2] += c->quad[2] + m * (3.0 * dv[0] * dv[2]);
    q[3] += c->quad[3] + m * (3.0 * dv[1] * dv[1] - dd);
    q[4] += c->quad[4] + m * (3.0 * dv[1] * dv[2]);
    q[5] += c->quad[5] + m * (3.0 * dv[2] * dv[2] - dd);
  }
  for (a = 0; a < 3; ++a) p->com[a] = com[a];
  p->com[3] = M;
  for (a = 0; a < 6; ++a) p->quad[a] = q[a];
}

/*
 * Leaf-first build.  Arguments and output layout as tbo_build (without the DFS
 * permutation); stage_s [6] (may be NULL) receives the seconds of steps (i)
 * keys, (ii) sort, (iii) reorder, (iv) leaves with their moments, (v) parents
 * with their moments, and the copy into the (depth, key)-ordered output.
 */
int tbl_build(const float *pos, const float *mass, int64_t n, int32_t n_leaf, const double lo[3],
              double side, int32_t *perm, uint64_t *cell_key, uint8_t *cell_level,
              int32_t *cell_first, int32_t *cell_count, int32_t *child_ptr, double *com,
              double *quad, int64_t *level_offset, int64_t *n_cells, double *stage_s) {
  uint64_t *keys = NULL, *sk = NULL;
  tbl_pair *pairs = NULL;
  float *spos = NULL, *smass = NULL;
  tbl_list leaves[TBL_LEVELS], inner[TBL_LEVELS], level[TBL_LEVELS];
  int64_t i, k, off;
  int d, deepest = 0, rc = TBL_OK;
  double t0 = seconds(), t1;

  memset(leaves, 0, sizeof(leaves));
  memset(inner, 0, sizeof(inner));
  memset(level, 0, sizeof(level));
  if (stage_s)
    for (d = 0; d < 6; ++d) stage_s[d] = 0.0;
  if (n < 0 || n > 2147483647LL || n_leaf < 1 || !lo || !n_cells || !level_offset)
    return TBL_ERR_ARG;
  if (n > 0 && (!pos || !mass || !perm || !cell_key || !cell_level || !cell_first ||
                !cell_count || !child_ptr || !com || !quad))
    return TBL_ERR_ARG;
  for (i = 0; i < 3 * n; ++i)
    if (!isfinite(pos[i])) return TBL_ERR_NONFINITE;
  for (i = 0; i < n; ++i)
    if (!(mass[i] > 0.0f) || !isfinite(mass[i])) return TBL_ERR_MASS;
  for (d = 0; d <= TBL_LEVELS; ++d) level_offset[d] = 0;
  *n_cells = 0;
  if (n == 0) return TBL_OK;

  keys = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  sk = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  pairs = (tbl_pair *)malloc((size_t)n * sizeof(tbl_pair));
  spos = (float *)malloc((size_t)n * 3 * sizeof(float));
  smass = (float *)malloc((size_t)n * sizeof(float));
  if (!keys || !sk || !pairs || !spos || !smass) {
    rc = TBL_ERR_NOMEM;
    goto done;
  }

  /* (i) keys */
  rc = tbo_keys(pos, n, lo, side, NULL, keys);
  if (rc) {
    rc = rc == -2 ? TBL_ERR_BOX : TBL_ERR_ARG;
    goto done;
  }
  t1 = seconds();
  if (stage_s) stage_s[0] = t1 - t0;
  t0 = t1;

  /* (ii) sort (key, index) pairs */
  for (i = 0; i < n; ++i) {
    pairs[i].key = keys[i];
    pairs[i].idx = (int32_t)i;
  }
  qsort(pairs, (size_t)n, sizeof(tbl_pair), cmp_key_idx);
  for (i = 0; i < n; ++i) {
    perm[i] = pairs[i].idx;
    sk[i] = pairs[i].key;
  }
  t1 = seconds();
  if (stage_s) stage_s[1] = t1 - t0;
  t0 = t1;

  /* (iii) reorder */
  for (i = 0; i < n; ++i) {
    int32_t p = perm[i];
    spos[3 * i + 0] = pos[3 * (int64_t)p + 0];
    spos[3 * i + 1] = pos[3 * (int64_t)p + 1];
    spos[3 * i + 2] = pos[3 * (int64_t)p + 2];
    smass[i] = mass[p];
  }
  t1 = seconds();
  if (stage_s) stage_s[2] = t1 - t0;
  t0 = t1;

  /* (iv) leaves, one after another */
  k = 0;
  while (k < n) {
    int D = 0;
    uint64_t lk;
    tbl_cell *leaf;
    if (k > 0) D = min_depth(sk[k - 1], sk[k]);
    if (k + n_leaf < n) {
      int r = min_depth(sk[k], sk[k + n_leaf]);
      if (r > D) D = r;
    }
    if (D > TBL_MAX_DEPTH) D = TBL_MAX_DEPTH;
    lk = cell_key_of(sk[k], D);
    leaf = list_push(&leaves[D]);
    if (!leaf) {
      rc = TBL_ERR_NOMEM;
      goto done;
    }
    leaf->key = lk;
    leaf->first = k;
    leaf->child = -1;
    while (k < n && cell_key_of(sk[k], D) == lk) ++k;
    leaf->count = k - leaf->first;
    leaf_moments(leaf, D, spos, smass, lo, side);
    if (D > deepest) deepest = D;
  }
  t1 = seconds();
  if (stage_s) stage_s[3] = t1 - t0;
  t0 = t1;

  /* (v) parents, deepest depth first; level[d] receives the cells of depth d
   * in key order as the two sorted lists are consumed */
  for (d = deepest; d >= 0; --d) {
    int64_t a = 0, b = 0;
    tbl_cell *parent = NULL;
    uint64_t last = 0; /* keys are >= 1: no parent is open */
    while (a < leaves[d].n || b < inner[d].n) {
      tbl_cell src, *c;
      if (b >= inner[d].n || (a < leaves[d].n && leaves[d].v[a].key < inner[d].v[b].key))
        src = leaves[d].v[a++];
      else
        src = inner[d].v[b++];
      c = list_push(&level[d]);
      if (!c) {
        rc = TBL_ERR_NOMEM;
        goto done;
      }
      *c = src;
      if (d == 0) continue; /* the root has no parent */
      if ((c->key >> 3) != last) {
        if (parent) parent_moments(parent, d, &level[d].v[parent->child], side);
        parent = list_push(&inner[d - 1]);
        if (!parent) {
          rc = TBL_ERR_NOMEM;
          goto done;
        }
        last = c->key >> 3;
        parent->key = last;
        parent->first = c->first;
        parent->child = level[d].n - 1;
      }
      parent->nchild += 1;
      parent->count += c->count;
    }
    if (parent) parent_moments(parent, d, &level[d].v[parent->child], side);
  }
  if (level[0].n != 1 || level[0].v[0].count != n) {
    rc = TBL_ERR_INTERNAL;
    goto done;
  }
  t1 = seconds();
  if (stage_s) stage_s[4] = t1 - t0;
  t0 = t1;

  /* canonical (depth, key) output */
  off = 0;
  for (d = 0; d < TBL_LEVELS; ++d) {
    level_offset[d] = off;
    off += level[d].n;
  }
  level_offset[TBL_LEVELS] = off;
  for (d = 0; d < TBL_LEVELS; ++d) {
    for (i = 0; i < level[d].n; ++i) {
      const tbl_cell *c = &level[d].v[i];
      int64_t o = level_offset[d] + i;
      int a;
      cell_key[o] = c->key;
      cell_level[o] = (uint8_t)d;
      cell_first[o] = (int32_t)c->first;
      cell_count[o] = (int32_t)c->count;
      child_ptr[2 * o] = c->child < 0 ? -1 : (int32_t)(level_offset[d + 1] + c->child);
      child_ptr[2 * o + 1] = c->child < 0 ? 0 : c->nchild;
      for (a = 0; a < 4; ++a) com[4 * o + a] = c->com[a];
      for (a = 0; a < 6; ++a) quad[6 * o + a] = c->quad[a];
    }
  }
  *n_cells = off;
  if (stage_s) stage_s[5] = seconds() - t0;

done:
  for (d = 0; d < TBL_LEVELS; ++d) {
    free(leaves[d].v);
    free(inner[d].v);
    free(level[d].v);
  }
  free(keys);
  free(sk);
  free(pairs);
  free(spos);
  free(smass);
  return rc;
}
