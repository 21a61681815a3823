/*
 * treebuild.h -- C ABI of the MI355X (gfx950) leaf-first oct-tree builder.
 *
 * The library builds the hashed oct-tree of Tokuue & Ishiyama (2023) on one GPU:
 *
 *   1. root box whose side is a power of two (Sec. 2.2);
 *   2. one 64-bit Morton key per particle: each coordinate quantised in FP64 to a
 *      21-bit integer, bits interleaved below a leading 1 (Sec. 2.2);
 *   3. a stable sort of (key, index) pairs; the index payload is `perm`
 *      (Sec. 2.3, steps ii-iii);
 *   4. every leaf straight from the sorted keys, with the leaf depth
 *      D_k = max(minDepth(k, k-1), minDepth(k, k+n_leaf)) of Sec. 2.3.1 and
 *      Appendix A, evaluated for all particles at once;
 *   5. the parents, one depth at a time from the deepest upwards, each created
 *      by the first of its children in key order and linked to all of them
 *      (Sec. 2.3.2, Algorithm 2);
 *   6. monopole, centre of mass and traceless quadrupole of every cell, leaves
 *      from their particles and parents from their children as soon as the
 *      children are complete (Sec. 2.3.2 and its footnotes).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named "device" are HIP device memory (e.g. PyTorch CUDA tensors);
 *   all of them are owned by the caller.  The library never allocates device
 *   memory on the build path; scratch space is the caller's `workspace`.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Builds are asynchronous: outputs are valid once the caller synchronises
 *   the stream.  A build performs no host/device synchronisation and no
 *   hipMemsetAsync, so a whole build may be captured into a hipGraph.
 * - Concurrent builds must use distinct workspaces and outputs.
 * - Return codes: TB_OK (0) or a negative TB_ERR_* value.  Host-detectable
 *   errors are returned synchronously before anything is launched.  Data errors
 *   found by kernels (non-finite position, non-positive mass) are OR-ed into
 *   the device status word `tb_tree.status` as bit flags; tb_build_sync() reads
 *   it back and returns the matching code.
 *
 * Key and cell layout
 * -------------------
 * - q_a = floor(fl64(x_a - lo_a) * 2^21 / side), clamped to [0, 2^21 - 1].
 *   Points outside the box are clamped into the edge cells.
 * - key = 2^63 | sum_b (qx_b << (3b+2) | qy_b << (3b+1) | qz_b << 3b), i.e. each
 *   3-bit octant digit is (x, y, z) with x most significant and 1 = upper half.
 * - A depth-d cell key is the upper 3d+1 bits of its particles' keys; the root
 *   key is 1.  Depths run from 0 to 21; a depth-21 leaf holds all particles
 *   with one key and may therefore exceed n_leaf.
 * - Cells are listed by (depth ascending, key ascending); cell 0 is the root.
 *   Children of a cell are contiguous at the next depth.
 * - Number of cells C <= C_max = N + 21 * floor(N / (n_leaf + 1)).
 *
 * Moment frames
 * -------------
 * - u = fl64(x - lo) is a particle's position in the box frame.  The centre of
 *   a depth-d cell with integer coordinates (i, j, k) is
 *   off = ((i, j, k) + 1/2) * side * 2^-d in that frame (exact).
 * - com[c] = {dx, dy, dz, M}: (dx, dy, dz) = sum m (u - off) / M, the centre of
 *   mass relative to the cell centre; M = sum m.
 * - quad[c] = {xx, xy, xz, yy, yz, zz} of Q_ab = sum m (3 r_a r_b - |r|^2 d_ab),
 *   r = u - off - (dx, dy, dz).  Q is traceless.
 * - TB_FP64: com and quad are double.  TB_MIXED: they are float, accumulated in
 *   FP32 with Kahan-compensated sums in cell-relative units; FP64 is used only
 *   for the quantisation and the root box.
 */
#ifndef TREEBUILD_H
#define TREEBUILD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TB_OK 0
#define TB_ERR_ARG (-1)       /* bad size, n_leaf, flag or NULL required pointer */
#define TB_ERR_BOX (-2)       /* side not a positive finite power of two, or lo not finite */
#define TB_ERR_WORKSPACE (-3) /* workspace NULL or smaller than tb_workspace_bytes() */
#define TB_ERR_HIP (-4)       /* a HIP runtime call failed */
#define TB_ERR_NONFINITE (-5) /* a position is NaN or infinite (device-detected) */
#define TB_ERR_MASS (-6)      /* a mass is not finite and positive (device-detected) */
#define TB_ERR_INTERNAL (-7)  /* a kernel found an inconsistent intermediate (a library bug) */
#define TB_ERR_SCRATCH (-8)   /* tb_build_noalloc: the build needs more than its fixed scratch */

/* Bits of the device status word. */
#define TB_STATUS_NONFINITE 1
#define TB_STATUS_MASS 2
#define TB_STATUS_INTERNAL 4 /* an index computed on the device fell out of range */
#define TB_STATUS_SETS 8     /* batch set offsets not 0 .. n_total and non-decreasing,
                                or a set larger than TB_SET_INDEX_BITS allows */
#define TB_STATUS_BOX 16     /* a batch box (device memory) failed the tb_box rules     */

/* Precision flags (bits 0..7). */
#define TB_FP64 0u
#define TB_MIXED 1u

/* Optional radix-sort shape in flag bits 8..15: an index into the table that
 * tb_sort_configs() lists; 0 is the default.  Every shape gives bit-identical
 * results; only speed and workspace size differ. */
#define TB_SORT_CONFIG(k) (((uint32_t)(k)&0xffu) << 8)

/* The radix passes of a single set of at least 512 sort tiles (about 2.9e6
 * particles with the default shape) normally take their tile offsets from a
 * separate count of every tile's digits (one byte an element, which the
 * previous pass leaves behind); smaller sets and batches use the decoupled
 * look-back across tiles.  This flag uses the look-back in every pass.  Results
 * are bit-identical either way; the flag exists for tuning and tests. */
#define TB_SORT_LOOKBACK (1u << 17)

/* Count the tiles' digits in every radix pass of any build, small sets and
 * batches too (a batch's offsets then start again at every set).  Not with
 * TB_SORT_LOOKBACK (TB_ERR_ARG).  Results are bit-identical. */
#define TB_SORT_COUNTED (1u << 19)

/* Build the cells subtree by subtree (Sec. 2.3.3, eq. 2): the sorted keys are
 * divided into blocks of at most 2048 particles that share no cell (the leaves
 * of the tree n_leaf = 2048 would give); one workgroup builds each block's
 * cells and moments with the leaf depth D_k = max(minDepth(k, k-1),
 * minDepth(k, k + n_leaf), d_root), d_root the block's depth; the cells above
 * the blocks are built from the block roots last.  Without the flag the cells
 * are placed tile by tile and the parents built one depth at a time over the
 * whole tree.  The tree is identical either way; only speed and workspace
 * differ. */
#define TB_SUBTREES (1u << 18)

/* Peano-Hilbert keys in place of Morton keys (footnote of Sec. 2.2).  The key
 * keeps its layout (a leading 1, then 21 3-bit digits), but the digits are the
 * index of the particle's depth-21 cell along the 3-D Hilbert curve of
 * Skilling's transpose method (J. Skilling, AIP Conf. Proc. 707, 381, 2004);
 * the curve starts at the box corner lo and steps between face neighbours, and
 * the top 3d bits of a key are the index of the depth-d cell on the d-level
 * curve, so cell keys are still prefixes of their particles' keys.  The cells,
 * their particles and moments are those of the Morton tree; cell_key holds the
 * Hilbert prefixes, cells and particles follow Hilbert order within a depth,
 * and a child's octant is no longer its key's last digit.  Pass the same bit
 * to tb_gravity for a tree built with it. */
#define TB_HILBERT (1u << 20)

/* A batch whose every set holds at most 2^k particles (k = 1 .. 31): the radix
 * sort carries each particle's index within its set (a batch sorts every set in
 * place) in k bits rather than its position in the batch, so that key and index
 * pack into one word earlier.  tb_build_batched only; a single build ignores
 * it.  A set larger than 2^k is reported as TB_STATUS_SETS (TB_ERR_ARG from the
 * _sync forms); the batch's outputs are then undefined (every set comes out as
 * a tree of coincident points), but every kernel stays inside its arrays.
 * Results are bit-identical with and without it. */
#define TB_SET_INDEX_BITS(k) ((((uint32_t)(k)) & 0x1fu) << 24)

#define TB_MAX_DEPTH 21
#define TB_MAX_NLEAF 1024 /* largest supported n_leaf */
#define TB_MAX_N 2147483647LL

typedef struct {
  double lo[3]; /* lower corner of the root cube */
  double side;  /* edge length: a positive power of two */
} tb_box;

/* Output buffers, all caller-owned DEVICE memory unless noted.  C_max is the
 * value returned by tb_max_cells(). */
typedef struct {
  int32_t *perm;         /* [N]        perm[s] = original index at sorted position s  */
  uint64_t *cell_key;    /* [C_max]    hashed oct-tree key                              */
  uint8_t *cell_level;   /* [C_max]    depth 0..21                                      */
  int32_t *cell_first;   /* [C_max]    first sorted position of the cell's particles    */
  int32_t *cell_count;   /* [C_max]    number of particles                              */
  int32_t *child_ptr;    /* [C_max][2] {first child cell, number of children}; {-1,0} leaf */
  void *com;             /* [C_max][4] double (TB_FP64) or float (TB_MIXED)              */
  void *quad;            /* [C_max][6] double (TB_FP64) or float (TB_MIXED)              */
  int64_t *level_offset; /* [23]       first cell of each depth; [22] = number of cells  */
  int64_t *n_cells;      /* [1]        number of cells                                   */
  int32_t *status;       /* [1]        OR of TB_STATUS_* bits; written by every build    */
  double *box_out;       /* [4] or NULL  the box used: lo[3], side                      */
  float *pos_sorted;     /* [N][3] or NULL  positions in sorted order (reorder, Sec. 2.3) */
  float *mass_sorted;    /* [N] or NULL     masses in sorted order                       */
  uint64_t *key_sorted;  /* [N] or NULL     particle keys in sorted order                */
} tb_tree;

/* C_max for N particles and leaf capacity n_leaf (0 for N = 0).
 * Errors: TB_ERR_ARG for N < 0, N > TB_MAX_N, n_leaf outside [1, TB_MAX_NLEAF]
 * or c_max == NULL. */
int tb_max_cells(int64_t n, int32_t n_leaf, int64_t *c_max);

/* Bytes of device workspace that tb_build() needs for these arguments.  On the
 * current device it also opts the cell kernels in to their full LDS size (a
 * per-device kernel attribute, set once per process); a caller that captures
 * builds into a HIP graph should size the workspace, or run one build, before
 * the capture, so that no attribute call happens inside it.
 * Errors: as tb_max_cells(), plus TB_ERR_ARG for unknown flags. */
int tb_workspace_bytes(int64_t n, int32_t n_leaf, uint32_t flags, size_t *bytes);

/* Build the tree of N particles (steps 1-6 above), asynchronously on `stream`.
 *   pos   [N][3] float, device, AoS (x, y, z)
 *   mass  [N]    float, device, finite and > 0
 *   box   host pointer; NULL = choose it from the data: lo = per-axis minimum,
 *         side = the smallest power of two strictly above the largest extent
 *         (1 if every extent is 0), computed in FP64 on the device
 *   flags TB_FP64 or TB_MIXED
 *   workspace / ws_bytes  device scratch of at least tb_workspace_bytes()
 *   out   host pointer to a tb_tree of device buffers (box_out, pos_sorted,
 *         mass_sorted, key_sorted may be NULL; the others are required when N > 0;
 *         level_offset, n_cells and status are required always)
 * Errors (synchronous): TB_ERR_ARG, TB_ERR_BOX, TB_ERR_WORKSPACE, TB_ERR_HIP. */
int tb_build(const float *pos, const float *mass, int64_t n, int32_t n_leaf, const tb_box *box,
             uint32_t flags, void *workspace, size_t ws_bytes, const tb_tree *out, void *stream);

/* tb_build() followed by a stream synchronisation and a read of the status
 * word; returns TB_ERR_NONFINITE or TB_ERR_MASS if the kernels flagged bad data. */
int tb_build_sync(const float *pos, const float *mass, int64_t n, int32_t n_leaf,
                  const tb_box *box, uint32_t flags, void *workspace, size_t ws_bytes,
                  const tb_tree *out, void *stream);

/* ------------------------------------------------------------------------- */
/* A build that allocates nothing, for callers that cannot allocate device
 * memory or pass a workspace: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, steps and results
 * as tb_build() without workspace / ws_bytes: the scratch space is a fixed
 * array of TB_NOALLOC_SCRATCH_BYTES in the library's device memory, one per
 * GPU, held from the first call on that GPU until the process ends.
 *   - The call allocates nothing (no hipMalloc, no hipFree, no allocating
 *     library routine) and performs no host synchronisation.
 *   - Every call on one GPU shares that GPU's array: calls that overlap in time
 *     on one GPU (two streams, two threads) race and give wrong results.
 *     Serialise them, e.g. on one stream.  The build clears what it needs
 *     cleared itself.
 *   - The caller still owns pos, mass and every output buffer of `out`.
 * Errors: as tb_build(), plus TB_ERR_SCRATCH (synchronous, before any launch)
 * when tb_workspace_bytes() for these arguments exceeds
 * TB_NOALLOC_SCRATCH_BYTES (64 MiB: about 10^6 particles at n_leaf 16). */
#define TB_NOALLOC_SCRATCH_BYTES (64u << 20)

int tb_build_noalloc(const float *pos, const float *mass, int64_t n, int32_t n_leaf,
                     const tb_box *box, uint32_t flags, const tb_tree *out, void *stream);

/* ------------------------------------------------------------------------- */
/* Batched builds: B independent particle sets in one sequence of launches.
 *
 * The sets are stored back to back: set b owns input particles
 * [set_offsets[b], set_offsets[b+1]) of pos / mass.  Each set gets its own tree,
 * exactly the tree tb_build() would give for that set alone (Sec. 2.3 applied
 * per set); the trees share the output arrays as follows:
 *   perm           set b's sorted positions are the same range
 *                  [set_offsets[b], set_offsets[b+1]); perm values stay global
 *                  input indices inside that range
 *   cells          set b's cells are the contiguous block
 *                  [cell_offsets[b], cell_offsets[b+1]), in (depth, key) order
 *                  within the block; cell_first and child_ptr hold global
 *                  sorted positions and global cell indices
 *   level_offset   [B][23]: row b = global first cell of each depth of set b,
 *                  [b][22] = cell_offsets[b+1]
 *   n_cells        total over all sets
 *   box_out        [B][4] or NULL
 * A set may be empty (no cells).  C_max = tb_max_cells(n_total, n_leaf) bounds
 * the total number of cells.
 *
 *   nsets        B, 1 .. TB_MAX_SETS
 *   set_offsets  [B+1] int64, DEVICE; 0 = set_offsets[0] <= ... <= set_offsets[B]
 *                = n_total.  Offsets that break this are reported on the device
 *                (TB_STATUS_SETS); the build then proceeds as one set, so no
 *                kernel reads outside [0, n_total).
 *   boxes        [B] tb_box, DEVICE, or NULL = each set's box from its own data
 *                (as tb_build() with box NULL).  A box that breaks the tb_box
 *                rules is reported (TB_STATUS_BOX) and replaced by the unit cube.
 *   cell_offsets [B+1] int64, DEVICE, or NULL.
 * Other arguments as tb_build(); the workspace size comes from
 * tb_workspace_bytes_batched().  A batch performs no host/device
 * synchronisation, so the whole batch may be captured into one hipGraph.
 * Errors (synchronous): TB_ERR_ARG (also nsets outside 1..TB_MAX_SETS or
 * set_offsets NULL), TB_ERR_WORKSPACE, TB_ERR_HIP. */
#define TB_MAX_SETS 16383

int tb_workspace_bytes_batched(int64_t n_total, int32_t nsets, int32_t n_leaf, uint32_t flags,
                               size_t *bytes);

int tb_build_batched(const float *pos, const float *mass, int64_t n_total, int32_t nsets,
                     const int64_t *set_offsets, int32_t n_leaf, const tb_box *boxes,
                     uint32_t flags, void *workspace, size_t ws_bytes, const tb_tree *out,
                     int64_t *cell_offsets, void *stream);

/* tb_build_batched() followed by a stream synchronisation and a read of the
 * status word: TB_ERR_NONFINITE, TB_ERR_MASS, TB_ERR_ARG (TB_STATUS_SETS) or
 * TB_ERR_BOX (TB_STATUS_BOX) if the kernels flagged the data. */
int tb_build_batched_sync(const float *pos, const float *mass, int64_t n_total, int32_t nsets,
                          const int64_t *set_offsets, int32_t n_leaf, const tb_box *boxes,
                          uint32_t flags, void *workspace, size_t ws_bytes, const tb_tree *out,
                          int64_t *cell_offsets, void *stream);

/* ------------------------------------------------------------------------- */
/* Gravity on the tree (Sec. 2.1): Barnes-Hut accelerations and potentials of
 * every particle, G = 1, from an FP64 tree that tb_build() made.
 *
 * Groups (Barnes' modified algorithm, Sec. 2.1): going down from the root, the
 * first cell on each path that holds at most n_crit particles, or is a leaf, is
 * a group, and its particles share one interaction list.  A cell C is accepted
 * for group G when it is neither G nor an ancestor of G and l_C < theta * d
 * (eq. 1), d the distance from C's centre of mass to the closest point of G's
 * cube; otherwise it is opened: a leaf contributes its particles, an internal
 * cell its children.  Terms, with r = x_i - x_C:
 *   accepted cell  phi = -M / r - (r.Q.r) / (2 r^5),
 *                  a = -M r / r^3 + Q r / r^5 - 5/2 (r.Q.r) r / r^7
 *                  (the Q terms with TB_GRAV_QUADRUPOLE, else monopole only);
 *   particle j     phi = -m_j / s, a = -m_j (x_i - x_j) / s^3,
 *                  s = (|x_i - x_j|^2 + eps^2)^(1/2), j != i.
 * Evaluated in FP64.
 *
 *   pos_sorted, mass_sorted  [N][3], [N] float, DEVICE: the particles in key
 *               order (tb_build's pos_sorted / mass_sorted outputs)
 *   tree        host pointer to the tb_tree of that build (TB_FP64 moments);
 *               box_out must have been filled; n_cells is read on the device
 *   c_max       tb_max_cells() of that build (bounds the cells examined)
 *   theta       opening angle (>= 0; 0 opens everything: direct summation)
 *   n_crit      group size (>= 1)
 *   eps         Plummer softening of the particle terms (>= 0)
 *   flags       0 or TB_GRAV_QUADRUPOLE, plus TB_HILBERT for a tree built on
 *               Peano-Hilbert keys
 *   acc         [N][4] double, DEVICE, out: ax, ay, az, phi in key order
 *   stats       [2] int64, DEVICE, or NULL: number of groups, and number of
 *               interactions (cell terms plus particle pairs) over all particles
 *   workspace   DEVICE, at least tb_gravity_workspace_bytes(c_max) bytes
 * Asynchronous on `stream`.  A group whose walk outgrows the kernel's 4096-cell
 * LDS stack sets TB_STATUS_INTERNAL in tree->status.
 * Errors (synchronous): TB_ERR_ARG, TB_ERR_WORKSPACE, TB_ERR_HIP. */
#define TB_GRAV_QUADRUPOLE 1u

int tb_gravity_workspace_bytes(int64_t c_max, size_t *bytes);

int tb_gravity(const float *pos_sorted, const float *mass_sorted, int64_t n, const tb_tree *tree,
               int64_t c_max, double theta, int32_t n_crit, double eps, uint32_t flags,
               double *acc, int64_t *stats, void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------- */
/* Particle updates of an N-body run around the build (Sec. 3: a leapfrog over
 * constant timesteps with the tree rebuilt every step; Sec. 2.3 and Sec. 4:
 * reordering the particles in memory is optional and may be done only every
 * few steps).
 *
 * tb_kick_drift: for every sorted position s, with i = perm[s] (i = s when perm
 * is NULL), in this order
 *     vel[i] += acc[s] * dt_kick,   pos[i] += vel[i] * dt_drift,
 * each component updated in FP64 (one rounding per operation) and stored in
 * FP32.  perm [N] int32 DEVICE (a build's perm, or NULL); acc [N][4] double
 * DEVICE (tb_gravity's output; the 4th column is ignored); pos, vel [N][3]
 * float DEVICE, updated in place; status int32 DEVICE or NULL: an index out of
 * [0, N) is skipped and sets TB_STATUS_INTERNAL.  A kick-drift-kick leapfrog
 * is kick_drift(dt/2, dt) on the first step, kick_drift(dt, dt) after, and a
 * closing kick_drift(dt/2, 0).
 *
 * tb_permute: dst[s][k] = src[perm[s]][k] for rows of `width` 4-byte words
 * (1 <= width <= 64): reorders particle arrays into the key order of the build
 * that produced perm.  src and dst must not overlap.  Same status behaviour.
 *
 * Both are asynchronous on `stream`.  Errors (synchronous): TB_ERR_ARG (N out
 * of range, null pointers, non-finite steps, bad width), TB_ERR_HIP. */
int tb_kick_drift(const int32_t *perm, const double *acc, int64_t n, double dt_kick,
                  double dt_drift, float *pos, float *vel, int32_t *status, void *stream);
int tb_permute(const int32_t *perm, int64_t n, const void *src, int32_t width, void *dst,
               int32_t *status, void *stream);

/* ------------------------------------------------------------------------- */
/* Kernel timing.  When enabled, every kernel launch of a build is bracketed by
 * HIP events recorded on the build's stream; the per-kernel durations are
 * summed when tb_trace_read() is called (which synchronises on the events).
 * Tracing is process-wide and not thread-safe; it is meant for benchmarks.   */
typedef struct {
  char name[48];     /* kernel name */
  int64_t launches;  /* number of launches recorded */
  double total_ms;   /* summed event-to-event duration */
} tb_trace_entry;

int tb_trace_enable(int on);
/* Copy up to `cap` entries into `out` and set *count; resets the accumulators. */
int tb_trace_read(tb_trace_entry *out, int cap, int *count);

/* The selectable radix-sort shapes: desc[3k..3k+2] = {digit bits, keys per
 * thread, threads per workgroup} of TB_SORT_CONFIG(k).  With cap = 0 only
 * *count (the table size) is written. */
int tb_sort_configs(int32_t *desc, int cap, int *count);

/* Library version string, e.g. "treebuild 0.2 gfx950". */
const char *tb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TREEBUILD_H */
