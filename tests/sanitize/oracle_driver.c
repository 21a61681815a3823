/*
 * Test driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code only): builds trees, walks them and exercises the key helpers on
 * small adversarial sets, and exits non-zero on any error code or mismatch.  The
 * sanitizers turn any out-of-bounds access, leak or undefined operation into a
 * failure of their own.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int tbo_build_curve(const float *pos, const float *mass, int64_t n, int32_t n_leaf,
                    const double lo[3], double side, int curve, int32_t *perm, int32_t *dfs_perm,
                    uint64_t *cell_key, uint8_t *cell_level, int32_t *cell_first,
                    int32_t *cell_count, int32_t *child_ptr, double *com, double *quad,
                    int64_t *level_offset, int64_t *n_cells, double *stage_s);
int64_t tbo_max_cells(int64_t n, int32_t n_leaf);
int tbl_build(const float *pos, const float *mass, int64_t n, int32_t n_leaf, const double lo[3],
              double side, int32_t *perm, uint64_t *cell_key, uint8_t *cell_level,
              int32_t *cell_first, int32_t *cell_count, int32_t *child_ptr, double *com,
              double *quad, int64_t *level_offset, int64_t *n_cells, double *stage_s);
int tbg_direct(const float *pos, const float *mass, int64_t n, double eps, double *acc);
int tbg_walk_tree_curve(const float *pos, const float *mass, const int32_t *perm, int64_t n,
                        const uint64_t *cell_key, const uint8_t *cell_level,
                        const int32_t *cell_first, const int32_t *cell_count,
                        const int32_t *child_ptr, const double *com, const double *quad,
                        const double lo[3], double side, double theta, int32_t n_crit,
                        double eps, int quad_on, int curve, double *acc, int64_t *stats);
void tbo_hilbert_encode(const uint32_t *q, int64_t n, int bits, uint64_t *h);
void tbo_hilbert_decode(const uint64_t *h, int64_t n, int bits, uint32_t *q);
int tbo_auto_box(const float *pos, int64_t n, double lo[3], double *side);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform01(void) { /* splitmix64 */
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(const char *name, const float *pos, const float *mass, int64_t n, int nl,
                    int curve) {
  const double lo[3] = {0.0, 0.0, 0.0};
  const int64_t cmax = tbo_max_cells(n, nl) + 1;
  int32_t *perm = malloc(sizeof(int32_t) * (n + 1)), *dfs = malloc(sizeof(int32_t) * (n + 1));
  uint64_t *key = malloc(sizeof(uint64_t) * cmax), *key2 = malloc(sizeof(uint64_t) * cmax);
  uint8_t *lvl = malloc(cmax), *lvl2 = malloc(cmax);
  int32_t *first = malloc(4 * cmax), *cnt = malloc(4 * cmax), *child = malloc(8 * cmax);
  int32_t *first2 = malloc(4 * cmax), *cnt2 = malloc(4 * cmax), *child2 = malloc(8 * cmax);
  int32_t *perm2 = malloc(sizeof(int32_t) * (n + 1));
  double *com = malloc(32 * cmax), *quad = malloc(48 * cmax), *com2 = malloc(32 * cmax),
         *quad2 = malloc(48 * cmax), *acc = malloc(40 * (n + 1)), stage[6];
  int64_t loff[23], loff2[23], nc = 0, nc2 = 0, stats[2];
  int rc = tbo_build_curve(pos, mass, n, nl, lo, 1.0, curve, perm, dfs, key, lvl, first, cnt,
                           child, com, quad, loff, &nc, stage);
  int bad = rc != 0;
  if (!bad && curve == 0) {
    rc = tbl_build(pos, mass, n, nl, lo, 1.0, perm2, key2, lvl2, first2, cnt2, child2, com2, quad2,
                   loff2, &nc2, stage);
    bad = rc != 0 || nc2 != nc || memcmp(perm, perm2, sizeof(int32_t) * n) != 0 ||
          memcmp(key, key2, sizeof(uint64_t) * nc) != 0 ||
          memcmp(child, child2, 8 * nc) != 0;
  }
  if (!bad && n > 0) {
    rc = tbg_walk_tree_curve(pos, mass, perm, n, key, lvl, first, cnt, child, com, quad, lo, 1.0,
                             0.6, 16, 1e-3, 1, curve, acc, stats);
    bad = rc != 0;
  }
  printf("%-24s curve=%d n=%lld n_leaf=%d cells=%lld %s\n", name, curve, (long long)n, nl,
         (long long)nc, bad ? "FAILED" : "ok");
  free(perm); free(dfs); free(key); free(key2); free(lvl); free(lvl2); free(first); free(cnt);
  free(child); free(first2); free(cnt2); free(child2); free(perm2); free(com); free(quad);
  free(com2); free(quad2); free(acc);
  return bad;
}

int main(void) {
  enum { N = 3000 };
  static float pos[3 * N], mass[N];
  int fails = 0, i, curve;
  for (i = 0; i < N; ++i) {
    pos[3 * i] = (float)uniform01();
    pos[3 * i + 1] = (float)uniform01();
    pos[3 * i + 2] = (float)uniform01();
    mass[i] = (float)(0.5 + uniform01());
  }
  for (curve = 0; curve <= 1; ++curve) {
    fails += run_case("uniform", pos, mass, N, 8, curve);
    fails += run_case("n_leaf 1", pos, mass, 500, 1, curve);
    fails += run_case("n = n_leaf", pos, mass, 16, 16, curve);
    fails += run_case("single", pos, mass, 1, 4, curve);
    fails += run_case("empty", pos, mass, 0, 4, curve);
  }
  /* duplicates and a saturated depth-21 leaf */
  for (i = 0; i < N; ++i) {
    const int b = i % 37;
    pos[3 * i] = (float)(0.1 + 0.02 * b);
    pos[3 * i + 1] = (float)(0.3 + 0.01 * b);
    pos[3 * i + 2] = (i < 100) ? 0.7f : (float)(0.2 + 0.015 * b);
  }
  for (curve = 0; curve <= 1; ++curve) fails += run_case("duplicates", pos, mass, N, 4, curve);
  /* points outside the box clamp into the edge cells */
  for (i = 0; i < N; ++i) {
    pos[3 * i] = (float)(1.6 * uniform01() - 0.3);
    pos[3 * i + 1] = (float)(1.6 * uniform01() - 0.3);
    pos[3 * i + 2] = (float)(1.6 * uniform01() - 0.3);
  }
  fails += run_case("outside box", pos, mass, N, 8, 0);
  {
    double lo[3], side;
    double *acc = malloc(sizeof(double) * 4 * 300);
    fails += tbo_auto_box(pos, N, lo, &side) != 0;
    fails += tbg_direct(pos, mass, 300, 1e-3, acc) != 0;
    free(acc);
  }
  {
    uint32_t q[3 * 512], q2[3 * 512];
    uint64_t h[512];
    for (i = 0; i < 512; ++i) {
      q[3 * i] = (uint32_t)(i & 7);
      q[3 * i + 1] = (uint32_t)((i >> 3) & 7);
      q[3 * i + 2] = (uint32_t)(i >> 6);
    }
    tbo_hilbert_encode(q, 512, 3, h);
    tbo_hilbert_decode(h, 512, 3, q2);
    fails += memcmp(q, q2, sizeof(q)) != 0;
  }
  printf("%s\n", fails ? "SANITIZED RUN FAILED" : "SANITIZED RUN OK");
  return fails ? 1 : 0;
}
