// tb_sort.hip -- stable LSD radix sort of (key, index) pairs (Sec. 2.3, step ii).
//
// One kernel launch per digit pass ("onesweep" structure):
//   * every workgroup takes the next tile of keys (dynamic tile id, so all
//     earlier tiles are already running and the look-back always progresses);
//   * each wave ranks its keys with 64-lane ballots: for every digit bit a
//     ballot, folded into the mask of lanes holding the same digit, whose
//     population below the lane is the lane's rank among equal digits; items
//     are processed in index order, so the ranking is stable;
//   * per-wave digit counts are combined in LDS; the tile publishes its
//     per-digit counts, then looks back over earlier tiles (decoupled look-back)
//     for its global exclusive prefix;
//   * keys and payloads are first sorted by digit inside the tile in LDS, then
//     written so that consecutive lanes store consecutive addresses of a digit
//     run.
// The global digit counts come from the key-generation pass (and become each
// digit's base once per build), so the keys are read only once per pass.  The
// index payload of the last pass is `perm`.
//
// By default the passes of a single set are "counted" instead (reduce, then
// scan; a batch with TB_SORT_COUNTED too): a first kernel reads each element's
// digit (one byte, left behind by the previous pass or the key kernel) and
// writes every tile's digit counts, a second turns them into exclusive
// prefixes over the tiles, and the scatter kernel reads its tile's offsets
// instead of waiting on its predecessors.  Reading that byte again costs less
// than the look-back chain across the chip; TB_SORT_LOOKBACK keeps the
// look-back.
//
// A batch sorts every set in place: a set's tiles never straddle it, its tiles'
// look-back chain starts at its own first tile, and its digit runs start at
// bases taken from its own digit counts (counted per set by the key kernel).
// The passes thus give the (set, key) order with no pass over the set id.
//
// Elements shrink as the passes go: a pass carries only the key bits later
// passes still need.  The first passes move the 64-bit key and the index in two
// arrays (12 bytes); once the key bits left fit beside the index in 64 or 32
// bits, both travel as one packed word, (key >> consumed bits) << idx_bits |
// index, whose digit is read at bit idx_bits.  The last pass writes the index
// alone.  The sorted keys themselves are recomputed from the sorted particles in
// the reorder pass, which reads those particles anyway.
#include "tb_internal.h"

namespace tb {

template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t *s_tmp,
                                                        uint32_t *total) {
  constexpr int WAVES = THREADS / 64;
  const int wv = threadIdx.x / 64;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane_id() == 63) s_tmp[wv] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < WAVES; ++k) {
    const uint32_t t = s_tmp[k];
    off += (k < wv) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Word type of an element format (kFormIdx and kFormPack32: 32-bit words).
template <int F>
struct FormType {
  using T = uint32_t;
};
template <>
struct FormType<kFormKey64> {
  using T = uint64_t;
};
template <>
struct FormType<kFormPack64> {
  using T = uint64_t;
};

// Digit at bit offset `shift` (uniform): the pass's digit position for a 64-bit
// key, idx_bits for a packed element.
template <int BITS>
__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift) {
  const uint32_t lo = (uint32_t)k, hi = (uint32_t)(k >> 32);
  const uint32_t w = shift < 32 ? __builtin_amdgcn_alignbit(hi, lo, (uint32_t)shift)
                                : (hi >> (shift - 32));
  return w & ((1u << BITS) - 1u);
}
template <int BITS>
__device__ __forceinline__ uint32_t digit_of(uint32_t k, int shift) {
  return (k >> shift) & ((1u << BITS) - 1u);
}

// Tiles of a pass.  A single set: tile t holds keys [t TILE, (t+1) TILE) of the
// array, and the digit runs start where the global digit counts put them.  A
// batch: every set is sorted in place; a set's tiles never straddle it, tile t
// of set b holds the set's keys [t TILE, (t+1) TILE) counted from the set's
// first tile, and each digit's run of the set starts at the set's own base.
struct SegTiles {
  const int64_t *tile_start;  // [B + 1] first tile of each set, or NULL (single set)
  const int32_t *tile_set;    // [tiles] set of each tile
  const int64_t *set_off;     // [B + 1] first position of each set
  size_t base_stride;         // words between two sets' rows of `hist`
  int32_t nsets;
};

// Digit counts of the tiles of a counted pass: tile t (its elements as the
// scatter kernel tiles them, SegTiles) gets cnt[d][t].  The digits come from
// dig, written for this pass by the key kernel (first pass) or by the previous
// pass's scatter, so a count reads one byte an element (two for 9-bit digits)
// instead of the element.  A workgroup counts TPW consecutive tiles at once
// (every thread's loads of all of them in flight together, one set of per-wave
// histograms per tile), which halves the waves for about the same wave life.
template <int BITS, int IPT, int THREADS, int TPW>
__global__ __launch_bounds__(THREADS) void k_tile_count(const void *__restrict__ dig_v, uint32_t n,
                                                        uint32_t *__restrict__ cnt,
                                                        uint32_t n_tiles, SegTiles seg) {
  using DT = DigitType<BITS>;
  constexpr int R = 1 << BITS;
  constexpr int WAVES = THREADS / 64;
  constexpr uint32_t TILE = (uint32_t)THREADS * IPT;
  __shared__ uint32_t h[TPW * WAVES * R];  // per tile, one histogram per wave
  for (int i = threadIdx.x; i < TPW * WAVES * R; i += THREADS) h[i] = 0;
  const DT *__restrict__ dig = static_cast<const DT *>(dig_v);
  const uint32_t t0 = blockIdx.x * TPW;
  const uint32_t tiles_here = seg.tile_start ? (uint32_t)seg.tile_start[seg.nsets] : n_tiles;
  uint32_t base[TPW], last[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const uint32_t tile = t0 + q;
    base[q] = tile * TILE;
    uint32_t hi = n;
    if (tile >= tiles_here) {  // past the last tile: counts nothing
      base[q] = 1u;
      hi = 1u;
    } else if (seg.tile_start) {
      const int b = seg.tile_set[tile];
      base[q] = (uint32_t)seg.set_off[b] + (uint32_t)((int64_t)(tile - seg.tile_start[b]) * TILE);
      hi = (uint32_t)seg.set_off[b + 1];
    }
    last[q] = min(base[q] + TILE, hi) - 1u;  // base[q] - 1 when the tile is empty
  }
  uint32_t k[TPW][IPT];
#pragma unroll
  for (int q = 0; q < TPW; ++q)
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      k[q][j] = dig[min(min(base[q] + j * THREADS + threadIdx.x, last[q]), n - 1u)];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    uint32_t *hw = h + (q * WAVES + threadIdx.x / 64) * R;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const bool valid = base[q] + j * THREADS + threadIdx.x <= last[q] &&
                         base[q] <= last[q];
      const uint32_t d = k[q][j];
      // clustered data gives few distinct digits per wave: groups of four or
      // more equal digits add once (all masks wave-uniform), the rest one by one
      uint64_t rem = __ballot(valid);
      while (rem != 0) {
        const int l = __builtin_ctzll(rem);
        const uint32_t d0 = __builtin_amdgcn_readlane(d, l);
        const uint64_t m = __ballot(d == d0) & rem;
        const uint32_t c = (uint32_t)__popcll(m);
        if (c < 4) break;
        if (lane_id() == l) atomicAdd(&hw[d0], c);
        rem &= ~m;
      }
      if ((rem >> lane_id()) & 1u) atomicAdd(&hw[d], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < TPW * R; i += THREADS) {
    const int q = i / R, d = i % R;
    if (t0 + q >= tiles_here) continue;
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) c += h[(q * WAVES + w) * R + d];
    cnt[(size_t)d * n_tiles + t0 + q] = c;
  }
}

// cnt[d][t] <- sum over t' < t of cnt[d][t']: one workgroup per digit, each
// thread a contiguous run of tiles.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_tile_scan(uint32_t *__restrict__ cnt,
                                                       uint32_t n_tiles) {
  __shared__ uint32_t s_tmp[THREADS / 64];
  uint32_t *row = cnt + (size_t)blockIdx.x * n_tiles;
  const uint32_t per = (n_tiles + THREADS - 1) / THREADS;
  const uint32_t t0 = min(threadIdx.x * per, n_tiles), t1 = min(t0 + per, n_tiles);
  uint32_t sum = 0;
  for (uint32_t t = t0; t < t1; ++t) sum += row[t];
  uint32_t total;
  uint32_t run = block_exclusive_sum<THREADS>(sum, s_tmp, &total);
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t c = row[t];
    row[t] = run;
    run += c;
  }
}


// All ones if bit b of d is set, else zero: one signed one-bit field extract
// (the compiler would otherwise shift left and then arithmetically right).
__device__ __forceinline__ uint32_t lane_bit_mask(uint32_t d, int b) {
  uint32_t m;
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(d), "i"(b));
  return m;
}

// Shape and LDS of one radix tile.  FIN / FOUT: element format read / written
// (FIN is never kFormIdx).
template <int BITS, int IPT, int THREADS, int FIN, int FOUT>
struct Sweep {
  using KI = typename FormType<FIN>::T;
  using KO = typename FormType<FOUT>::T;
  static constexpr bool PIN = FIN != kFormKey64;  // packed input: the index is in the word
  static constexpr int R = 1 << BITS;
  static constexpr int WAVES = THREADS / 64;
  static constexpr int TILE = THREADS * IPT;
  static constexpr int DPT = (R + THREADS - 1) / THREADS;  // digits per thread
  // the local sort keeps the input word, except where only a separate index is
  // written: there the digit of each slot suffices
  static constexpr bool SLOT_DIGIT = FOUT == kFormIdx && !PIN;
  static constexpr int SLOT_BYTES = SLOT_DIGIT ? 2 : (int)sizeof(KI);
  struct Lds {
    alignas(16) unsigned char slot[TILE * SLOT_BYTES];
    uint32_t vals[PIN ? 1 : TILE];
    uint32_t wc[WAVES * R];   // per-wave digit counters, then wave offsets
    uint32_t tstart[R];       // tile-local start of each digit
    int32_t goff[R];          // output position minus tile-local position
    uint32_t tmp[WAVES];
    uint32_t tile;
  };
};

// Wave-striped load of a tile: item j of lane l is element wbase + j*64, with
// wbase = lo + wave*64*IPT + l.  Loads are branch-free (indices past the tile
// are clamped and the items masked later) so that all of them are in flight
// together.  v: the separate index of kFormKey64; when vin is NULL, the position
// less vbase (the set's first position in a batch, whose sort carries indices
// within the set).
template <class S, int IPT>
__device__ __forceinline__ void sweep_load(const typename S::KI *__restrict__ kin,
                                           const uint32_t *__restrict__ vin, uint32_t wbase,
                                           uint32_t last, uint32_t vbase,
                                           typename S::KI (&k)[IPT], uint32_t (&v)[IPT]) {
#pragma unroll
  for (int j = 0; j < IPT; ++j) k[j] = kin[min(wbase + j * 64, last)];
  if constexpr (!S::PIN) {
    if (vin) {
#pragma unroll
      for (int j = 0; j < IPT; ++j) v[j] = vin[min(wbase + j * 64, last)];
    } else {
#pragma unroll
      for (int j = 0; j < IPT; ++j) v[j] = wbase + j * 64 - vbase;
    }
  }
}

// Ranks a loaded tile and sorts it by digit in LDS.  On entry L.wc is zero
// (behind a barrier).  On return, for each digit d = threadIdx.x * DPT + t:
// tcnt[t] its count in the tile and trun[t] its tile-local start; with PUBLISH
// the tile's per-digit counts are also published for the look-back (inclusive
// when it is the first tile of its set).
template <class S, int BITS, int IPT, int THREADS, bool PUBLISH>
__device__ __forceinline__ void sweep_rank(typename S::Lds &L, const typename S::KI (&k)[IPT],
                                           const uint32_t (&v)[IPT], uint32_t wbase,
                                           uint32_t last, int shift, uint64_t *status,
                                           uint32_t tile, bool first, uint32_t (&tcnt)[S::DPT],
                                           uint32_t (&trun_d)[S::DPT]) {
  constexpr int R = S::R, WAVES = S::WAVES, DPT = S::DPT;
  const int wv = threadIdx.x / 64;
  const uint64_t lt = lanemask_lt();
  uint32_t dg[IPT], rk[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) dg[j] = digit_of<BITS>(k[j], shift);

  // Stable wave-level ranking: for every digit bit a ballot; XNOR-ing the
  // ballot with "all ones if my bit is set" keeps exactly the lanes that agree
  // with me on that bit, so the AND over all bits is the set of lanes holding
  // my digit.  Its population below my lane is my rank among them.  (The mask
  // is a signed one-bit field extract, which also feeds the ballot, and each
  // half of the AND is one three-input bit operation: four instructions a bit.
  // The operation's table is indexed by (a, b, c) bits as a*4 + b*2 + c, so
  // a & ~(b ^ c) is 0xF0 & ~(0xCC ^ 0xAA) = 0x90.)
  uint32_t *wc = L.wc + wv * R;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const bool valid = wbase + j * 64 <= last;
    const uint32_t d = dg[j];
    const uint64_t vmask = __ballot(valid);
    uint32_t plo = (uint32_t)vmask, phi = (uint32_t)(vmask >> 32);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const uint32_t m = lane_bit_mask(d, b);  // bit b set: all ones
      const uint64_t bb = __ballot(m != 0u);
      plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)bb, m, 0x90);
      phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(bb >> 32), m, 0x90);
    }
    const uint64_t peers = ((uint64_t)phi << 32) | plo;
    const uint32_t pre = (uint32_t)__popcll(peers & lt);
    uint32_t cnt = 0;
    if (valid) cnt = wc[d];
    rk[j] = cnt + pre;
    if (valid && pre == 0) wc[d] = cnt + (uint32_t)__popcll(peers);
  }
  __syncthreads();

  // per digit: exclusive offsets across waves and the tile count
#pragma unroll
  for (int t = 0; t < DPT; ++t) {
    const int d = threadIdx.x * DPT + t;
    uint32_t run = 0;
    if (d < R) {
#pragma unroll
      for (int q = 0; q < WAVES; ++q) {
        const uint32_t c = L.wc[q * R + d];
        L.wc[q * R + d] = run;
        run += c;
      }
      if constexpr (PUBLISH)
        atomic_store_agent(&status[(size_t)tile * R + d],
                           (first ? kFlagInclusive : kFlagAggregate) | (uint64_t)run);
    }
    tcnt[t] = run;
  }

  // tile-local digit starts: a block scan over the digits
  uint32_t tsum = 0;
#pragma unroll
  for (int t = 0; t < DPT; ++t) tsum += tcnt[t];
  uint32_t dummy;
  uint32_t trun = block_exclusive_sum<THREADS>(tsum, L.tmp, &dummy);
#pragma unroll
  for (int t = 0; t < DPT; ++t) {
    const int d = threadIdx.x * DPT + t;
    if (d < R) L.tstart[d] = trun;
    trun_d[t] = trun;
    trun += tcnt[t];
  }
  __syncthreads();

  // sort the tile by digit in LDS (the input word, or the digit where only a
  // separate index is written)
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if (wbase + j * 64 <= last) {
      const uint32_t d = dg[j];
      const uint32_t p = L.tstart[d] + wc[d] + rk[j];
      if constexpr (S::SLOT_DIGIT)
        reinterpret_cast<uint16_t *>(L.slot)[p] = (uint16_t)d;
      else
        reinterpret_cast<typename S::KI *>(L.slot)[p] = k[j];
      if constexpr (!S::PIN) L.vals[p] = v[j];
    }
  }
}

// Coalesced scatter of a tile sorted in LDS (L.goff set, behind a barrier):
// consecutive lanes write consecutive slots of a digit run, inside [set_lo, hi).
// A packed output word holds the key bits above this digit over the index; the
// last pass writes the index plus set_lo (a batch's indices are within the set).
// dig_out (a counted next pass): the next pass's digit of each element, at its
// output position.
template <class S, int BITS, int THREADS, int FOUT>
__device__ __forceinline__ void sweep_scatter(const typename S::Lds &L, uint32_t tile_n, int shift,
                                              int ib, uint32_t set_lo, uint32_t hi,
                                              typename S::KO *__restrict__ kout,
                                              uint32_t *__restrict__ vout,
                                              DigitType<BITS> *__restrict__ dig_out, bool &bad) {
  using KI = typename S::KI;
  using KO = typename S::KO;
  const uint32_t idx_mask = ib >= 32 ? 0xffffffffu : (1u << ib) - 1u;
  for (uint32_t i = threadIdx.x; i < tile_n; i += THREADS) {
    uint32_t d;
    KI kk = 0;
    if constexpr (S::SLOT_DIGIT) {
      d = reinterpret_cast<const uint16_t *>(L.slot)[i];
    } else {
      kk = reinterpret_cast<const KI *>(L.slot)[i];
      d = digit_of<BITS>(kk, shift);
    }
    const uint32_t idx = S::PIN ? ((uint32_t)kk & idx_mask) : L.vals[i];
    const uint32_t gp = (uint32_t)(L.goff[d] + (int32_t)i);
    if (gp < set_lo || gp >= hi) {  // cannot happen with consistent digit counts
      bad = true;
      continue;
    }
    if constexpr (FOUT == kFormIdx) {
      vout[gp] = idx + set_lo;
    } else {
      // the key bits above this digit: the next pass's digit at their bottom
      const uint64_t rest = (uint64_t)kk >> (shift + BITS);
      if constexpr (FOUT == kFormKey64) {
        kout[gp] = (KO)kk;
        vout[gp] = idx;
      } else {
        kout[gp] = (KO)((rest << ib) | idx);
      }
      if (dig_out) dig_out[gp] = (DigitType<BITS>)(rest & ((1u << BITS) - 1u));
    }
  }
}

// One radix pass, one workgroup per tile.  kin/kout hold the key or packed
// words; vin/vout the separate index of kFormKey64 (vin NULL: the index is the
// position) and the output of kFormIdx.  shift: the digit's bit offset in the
// input word; ib: idx_bits.  hist: the pass's digit bases, where each digit's
// run starts in the output [radix]; a batch has a row per set (set b at b *
// base_stride).
//
// Waves a SIMD a pass's registers must allow (the second launch bound; 1: no
// limit).  With 8-bit digits a pass over 32-bit packed words needs little LDS,
// so held to six waves (80 VGPRs, a 12-byte spill a lane) it runs three
// 512-thread workgroups a CU instead of two: 47.6 -> 43.8 us at 2^24.  So does
// a batch's look-back pass over 64-bit packed words with 5120-key tiles (a
// 28-byte spill; the 4096-set batch's sort 6.45 -> 6.34 ms), while the counted
// single-set pass loses more to its spill than it gains (sort 0.79 -> 0.87 ms)
// and larger tiles leave no LDS for a third workgroup.
template <int BITS, int IPT, int THREADS, int FIN, bool COUNTED, bool SEG>
constexpr int sweep_waves() {
  if (BITS != 8) return 1;
  if (FIN == kFormPack32) return 6;
  if (FIN == kFormPack64 && SEG && !COUNTED && THREADS == 512 && THREADS * IPT <= 5120) return 6;
  return 1;
}

template <int BITS, int IPT, int THREADS, int FIN, int FOUT, bool COUNTED, bool SEG>
__global__ __launch_bounds__(THREADS, (sweep_waves<BITS, IPT, THREADS, FIN, COUNTED, SEG>())) void k_onesweep(
    const void *__restrict__ kin_v, void *__restrict__ kout_v,
    const uint32_t *__restrict__ vin, uint32_t *__restrict__ vout, uint32_t n, int shift,
    int ib, const uint32_t *__restrict__ hist, uint64_t *__restrict__ status,
    uint64_t *__restrict__ status_next, uint32_t *__restrict__ tile_counter,
    const uint32_t *__restrict__ tile_off, int32_t *__restrict__ status_word, uint32_t n_tiles,
    SegTiles seg, void *__restrict__ dig_out) {
  using S = Sweep<BITS, IPT, THREADS, FIN, FOUT>;
  using KI = typename S::KI;
  constexpr int R = S::R, WAVES = S::WAVES, TILE = S::TILE, DPT = S::DPT;
  __shared__ typename S::Lds L;
  const KI *__restrict__ kin = static_cast<const KI *>(kin_v);
  typename S::KO *__restrict__ kout = static_cast<typename S::KO *>(kout_v);
  constexpr bool batch = SEG;

  // Look-back passes take tiles in the order they start, so that every earlier
  // tile is already running; counted passes need no order.
  if (!COUNTED && threadIdx.x == 0) L.tile = atomicAdd(tile_counter, 1u);
  for (int i = threadIdx.x; i < WAVES * R; i += THREADS) L.wc[i] = 0;
  __syncthreads();
  const uint32_t tile = COUNTED ? xcd_tile(blockIdx.x, gridDim.x) : L.tile;
  // a batch launches one workgroup for each tile it may have
  const uint32_t tiles_here = batch ? (uint32_t)seg.tile_start[seg.nsets] : n_tiles;
  if (tile >= tiles_here) {
    // a single set launches one workgroup per tile: the counter was not reset
    if (!batch && threadIdx.x == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
    return;
  }
  // the tile's elements [lo, lo + tile_n); its set's first tile starts the look-back
  uint32_t lo = tile * (uint32_t)TILE, hi = n, set_lo = 0u, set_tile0 = 0u;
  bool first = tile == 0;
  const uint32_t *digit_base = hist;
  if constexpr (batch) {
    const int b = seg.tile_set[tile];
    const int64_t t0 = seg.tile_start[b];
    set_tile0 = (uint32_t)t0;
    set_lo = (uint32_t)seg.set_off[b];
    lo = set_lo + (uint32_t)((int64_t)(tile - t0) * TILE);
    hi = (uint32_t)seg.set_off[b + 1];
    first = (int64_t)tile == t0;
    digit_base = hist + (size_t)b * seg.base_stride;
  }
  const uint32_t tile_n = (hi - lo) < (uint32_t)TILE ? (hi - lo) : (uint32_t)TILE;
  const uint32_t last = lo + tile_n - 1u;
  // where each digit's run starts does not depend on the elements: load it first
  uint32_t g[DPT];
#pragma unroll
  for (int t = 0; t < DPT; ++t) {
    const int d = threadIdx.x * DPT + t;
    g[t] = (d < R) ? digit_base[d] : 0u;
  }
  const uint32_t wbase = lo + (uint32_t)(threadIdx.x / 64) * 64u * IPT + (uint32_t)lane_id();
  KI k[IPT];
  uint32_t v[IPT];
  sweep_load<S, IPT>(kin, vin, wbase, last, set_lo, k, v);

  uint32_t tcnt[DPT], trun_d[DPT];
  sweep_rank<S, BITS, IPT, THREADS, !COUNTED>(L, k, v, wbase, last, shift, status, tile, first,
                                               tcnt, trun_d);
  // where each digit's run starts in the output: g, the pass's digit bases
  // the next pass's look-back words for this tile start cleared
  for (int i = threadIdx.x; i < R; i += THREADS) status_next[(size_t)tile * R + i] = 0;

  // the counted offsets (or the decoupled look-back within the set), one thread per digit
#pragma unroll
  for (int t = 0; t < DPT; ++t) {
    const int d = threadIdx.x * DPT + t;
    if (d < R) {
      uint32_t excl = 0;
      if (COUNTED) {
        // the prefix over all earlier tiles, less the prefix before the set's first tile
        excl = tile_off[(size_t)d * n_tiles + tile];
        if (batch) excl -= tile_off[(size_t)d * n_tiles + set_tile0];
      } else if (!first) {
        bool timed_out = false;
        excl = lookback<2>(status, R, tile, d, timed_out);
        if (timed_out) atomicOr(status_word, TB_STATUS_INTERNAL);
        atomic_store_agent(&status[(size_t)tile * R + d],
                           kFlagInclusive | (uint64_t)(excl + tcnt[t]));
      }
      L.goff[d] = (int32_t)(g[t] + excl - trun_d[t]);
    }
  }
  __syncthreads();

  bool bad = false;
  sweep_scatter<S, BITS, THREADS, FOUT>(L, tile_n, shift, ib, set_lo, hi, kout, vout,
                                        static_cast<DigitType<BITS> *>(dig_out), bad);
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
}

template <int BITS, int IPT, int THREADS, int FIN, int FOUT, bool COUNTED>
static hipError_t launch_pass_k(const Plan &p, const Work &w, int pass, const tb_tree &out,
                                hipStream_t s) {
  const int P = p.key_passes;
  void *K[2] = {w.keys0, w.keys1};
  // the last pass must write its index into out.perm
  uint32_t *V[2];
  V[P % 2] = reinterpret_cast<uint32_t *>(out.perm);
  V[(P + 1) % 2] = w.vals1;
  uint64_t *S[2] = {w.status0, w.status1};
  const uint32_t *vin = (pass == 0 || FIN != kFormKey64) ? nullptr : V[pass % 2];
  const int R = 1 << BITS;
  const int shift = FIN == kFormKey64 ? pass * BITS : p.idx_bits;
  SegTiles seg{nullptr, nullptr, nullptr, 0, p.nsets};
  const uint32_t *hist = w.hist + (size_t)pass * R;
  if (p.seg) {
    seg = SegTiles{w.seg_tile_start, w.seg_tile_set, w.set_off, (size_t)p.key_passes * R,
                   p.nsets};
    hist = w.seg_base + (size_t)pass * R;
  }
  if constexpr (COUNTED) {
    constexpr int TPW = 2;
    k_tile_count<BITS, IPT, THREADS, TPW>
        <<<(unsigned)((p.sort_tiles + TPW - 1) / TPW), THREADS, 0, s>>>(
            w.dig, (uint32_t)p.n, w.tile_off, (uint32_t)p.sort_tiles, seg);
    // tiles past the batch's last one count nothing and come after every real
    // tile, so the scan's prefixes for the real tiles are unaffected
    k_tile_scan<1024><<<R, 1024, 0, s>>>(w.tile_off, (uint32_t)p.sort_tiles);
  }
  // a counted pass that follows needs this pass to leave its digits behind
  void *dig_out = (pass + 1 < P && ((p.counted >> (pass + 1)) & 1u)) ? w.dig : nullptr;
  auto k = p.seg ? k_onesweep<BITS, IPT, THREADS, FIN, FOUT, COUNTED, true>
                 : k_onesweep<BITS, IPT, THREADS, FIN, FOUT, COUNTED, false>;
  k<<<(unsigned)p.sort_tiles, THREADS, 0, s>>>(
      K[pass % 2], K[(pass + 1) % 2], vin, V[(pass + 1) % 2], (uint32_t)p.n, shift, p.idx_bits,
      hist, S[pass % 2], S[(pass + 1) % 2], w.counters + pass, w.tile_off, out.status,
      (uint32_t)p.sort_tiles, seg, dig_out);
  return hipGetLastError();
}

template <int BITS, int IPT, int THREADS, int FIN, int FOUT>
static hipError_t launch_pass_c(const Plan &p, const Work &w, int pass, const tb_tree &out,
                                hipStream_t s) {
  return ((p.counted >> pass) & 1u)
             ? launch_pass_k<BITS, IPT, THREADS, FIN, FOUT, true>(p, w, pass, out, s)
             : launch_pass_k<BITS, IPT, THREADS, FIN, FOUT, false>(p, w, pass, out, s);
}

// The format pairs make_plan produces for 8- and 9-bit digits and any N below
// 2^32 (a 64-bit key is packed by the time 32 of its bits are consumed, since the
// 32 bits left and at most 32 index bits fit in 64).
template <int BITS, int IPT, int THREADS>
static hipError_t launch_pass_t(const Plan &p, const Work &w, int pass, const tb_tree &out,
                                hipStream_t s) {
  const int fi = p.form[pass], fo = p.form[pass + 1];
#define TB_PAIR(FI, FO) \
  if (fi == FI && fo == FO) return launch_pass_c<BITS, IPT, THREADS, FI, FO>(p, w, pass, out, s);
  TB_PAIR(kFormKey64, kFormKey64)
  TB_PAIR(kFormKey64, kFormPack64)
  TB_PAIR(kFormPack64, kFormPack64)
  TB_PAIR(kFormPack64, kFormPack32)
  TB_PAIR(kFormPack64, kFormIdx)
  TB_PAIR(kFormPack32, kFormPack32)
  TB_PAIR(kFormPack32, kFormIdx)
#undef TB_PAIR
  return hipErrorInvalidValue;
}

hipError_t launch_sort_pass(const Plan &p, const Work &w, int pass, const tb_tree &out,
                            hipStream_t s) {
  const SortConfig &c = p.sort;
#define TB_SORT_CASE(B, I, T)                                         \
  if (c.bits == B && c.ipt == I && c.threads == T)                    \
    return launch_pass_t<B, I, T>(p, w, pass, out, s);
  TB_SORT_CASE(8, 11, 512)
  TB_SORT_CASE(8, 12, 512)
  TB_SORT_CASE(8, 10, 512)
  TB_SORT_CASE(8, 16, 256)
  TB_SORT_CASE(9, 16, 256)
  TB_SORT_CASE(8, 12, 256)
  TB_SORT_CASE(8, 8, 512)
#undef TB_SORT_CASE
  return hipErrorInvalidValue;
}

bool sort_config_supported(const SortConfig &c) {
  static const int table[][3] = {{8, 11, 512}, {8, 12, 512}, {8, 10, 512}, {8, 16, 256},
                                 {9, 16, 256}, {8, 12, 256}, {8, 8, 512}};
  for (const auto &r : table)
    if (r[0] == c.bits && r[1] == c.ipt && r[2] == c.threads) return true;
  return false;
}

}  // namespace tb
