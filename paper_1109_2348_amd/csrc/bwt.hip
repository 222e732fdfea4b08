// Block BWT as a prefix-doubling sort of cyclic rotations (Sec. 3.1: the BWT
// is the sort of the rotations; Sec. 2.1: GPU sorting and lexicographic
// naming by prefix sums).
//
// All blocks of a batch share one array of SA rows (row k of block b lives at
// blk_off[b] + local row).  A rotation's rank is the row of the first member
// of its group ("head"), so ranks of different blocks never collide and rank
// order is rotation order.
//
//  init   rows start in descending start order; stable LSD radix per
//         block on the first INIT_BYTES cyclic bytes (big-endian); name
//         groups.  The first pass builds the (key, row) pairs from a
//         sequential read of the block's text; the others move them as plain
//         pairs, so no pass gathers at random.
//  round  for every unresolved group (a "segment"), key2 = rank of the
//         rotation h positions on (h = the prefix length the rotations are
//         ordered by); stable sort of the segment by key2; a new group
//         starts where key2 changes; rank = row of its head.  Groups of one
//         row are done; groups whose block length is <= the new prefix hold
//         equal rotations and are done too.  The prefix doubles.
//  round 0 (h = INIT_BYTES) takes key2 from the text instead: the 4 bytes
//         h positions on order those rotations exactly as their ranks would,
//         and they come from the block's L2-resident text (the prefix grows
//         by 4).  So the init naming ranks only the rows already alone in
//         their group, and round 0 ranks the rest.
//
// Stable sorts from a descending start order leave equal rotations in
// descending start order.  Segments of at most SMALL_MAX rows are packed into
// tiles and sorted in LDS; larger ones go through global LSD radix passes in
// which each segment keeps its own histogram column (a segmented sort).  The
// gather of key2 runs as its own kernel so that no rank is read after it has
// been refined in the same round.
#include <cstdio>
#include <algorithm>
#include <cstdlib>

#include "common.hpp"
#include "internal.hpp"
#include "plan.hpp"

namespace bzg {

constexpr int RI = RADIX_TILE / NT;  // 16 items per thread
constexpr int NW = NT / BZG_WAVE;    // 4 waves

__device__ __forceinline__ uint32_t find_block(const uint32_t* off, uint32_t nb, uint32_t k) {
  uint32_t lo = 0, hi = nb - 1;  // last b with off[b] <= k
  while (lo < hi) {
    uint32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t lowest_lane(uint64_t m) { return (uint32_t)(__ffsll((long long)m) - 1); }

// ------------------------------------------------------------------ init

// q mod n for q <= n + 2 and n >= 1 (a position at most 3 past the block
// end): three conditional subtractions cover even one-byte blocks.
__device__ __forceinline__ uint32_t cyc(uint32_t q, uint32_t n) {
  q = q >= n ? q - n : q;
  q = q >= n ? q - n : q;
  return q >= n ? q - n : q;
}

// The first 4 bytes of the rotation at local position pos, big-endian, in
// two steps, so that a caller issues the loads of all its rows before it
// uses any.  text_key_load reads the aligned dwords that hold bytes
// min(pos, n-4) .. +3 (one dword when that is aligned; each holds a byte of
// the block, so neither leaves the allocation's pages); text_key_value
// assembles them, or, for the few rotations that wrap around the block end
// (and blocks under 4 bytes), reads the 4 bytes one by one.
struct TextWords {
  uint32_t lo, hi;
};

__device__ __forceinline__ uint32_t text_key_addr(uint32_t o, uint32_t n, uint32_t pos) {
  return o + (n >= 4u ? min(pos, n - 4u) : 0u);
}

__device__ __forceinline__ TextWords text_key_load(const uint8_t* __restrict__ text, uint32_t o, uint32_t n,
                                                   uint32_t pos) {
  const uint32_t a = text_key_addr(o, n, pos);
  const uint32_t* w = (const uint32_t*)(text + (a & ~3u));
  TextWords t;
  t.lo = w[0];
  t.hi = w[(a & 3u) && n >= 4u ? 1 : 0];
  return t;
}

__device__ __forceinline__ uint32_t text_key_value(TextWords t, const uint8_t* __restrict__ text, uint32_t o,
                                                   uint32_t n, uint32_t pos) {
  if (pos + 3u < n) {
    const uint32_t sh = (text_key_addr(o, n, pos) & 3u) * 8u;
    return __builtin_bswap32(sh ? (t.lo >> sh) | (t.hi << (32u - sh)) : t.lo);
  }
  uint32_t v = 0;
#pragma unroll
  for (uint32_t j = 0; j < 4; j++) v = (v << 8) | text[o + cyc(pos + j, n)];
  return v;
}

// -------------------------------------------------- segment radix passes

struct BigTile {
  SegRec r;
  uint32_t t, nt, lo, hi;
};

__device__ __forceinline__ BigTile big_tile(uint32_t j, const SegRec* segs, const uint32_t* owner) {
  BigTile g;
  g.r = segs[owner[j]];
  g.nt = (g.r.len + RADIX_TILE - 1) / RADIX_TILE;
  g.t = j - g.r.base;
  g.lo = g.r.start + g.t * RADIX_TILE;
  g.hi = min(g.lo + RADIX_TILE, g.r.start + g.r.len);
  return g;
}

// Per-tile digit counts of one LSD pass: digit = (kin >> shift) & 255.
// The init sort orders rotations by their first INIT_BYTES bytes (one LSD
// pass each); the first doubling round then compares the 4 bytes after them
// in the text, so rotations are ordered by INIT_BYTES + 4 bytes after it.
// Four: with three, the pass saved (4.7 ms on 8192 uneven blocks) went back
// into the first round's larger groups (4.8 ms).
constexpr uint32_t INIT_BYTES = 4;
constexpr uint32_t INIT_MASK = 0xFFFFFFFFu << (8 * (4 - INIT_BYTES));  // the key bits the init sort orders

// INIT instantiates the init sort's passes (a kernel of their own for
// profiling); its first pass (text != null) reads the digit, byte
// INIT_BYTES - 1 of each row's first bytes, from the text instead (rows are
// in descending start order, so the read is sequential).  Init segments are
// whole blocks.
template <bool INIT>
__device__ void radix_hist_tile(uint32_t jt, const SegRec* __restrict__ segs, const uint32_t* __restrict__ owner,
                                const uint32_t* __restrict__ kin, int shift, uint32_t* __restrict__ hist,
                                const uint8_t* __restrict__ text) {
  // counts only (no ranks), so LDS atomics instead of matching lanes of
  // equal digit.  Same-address atomics serialize: every wave keeps 4 copies
  // (by lane mod 4, padded onto different banks), and the digit of each
  // slot's first lane, often the common one in skewed data, is added once
  // for all its lanes.
  constexpr uint32_t NC = NW * 4, CS = 257;
  __shared__ uint32_t cnt[NC * CS];
  const uint32_t w = threadIdx.x / BZG_WAVE;
  for (uint32_t d = threadIdx.x; d < NC * CS; d += NT) cnt[d] = 0;
  __syncthreads();
  BigTile g = big_tile(jt, segs, owner);
  const bool from_text = INIT && text != nullptr;
  const uint32_t wbase = g.lo + w * (RI * BZG_WAVE);
  // loads of clamped rows, none under a branch, so all are in flight at once
  uint32_t dg[RI];
  if (from_text) {
    const uint32_t o = g.r.start, n = g.r.len;
#pragma unroll
    for (int i = 0; i < RI; i++) {
      const uint32_t k = min(wbase + i * BZG_WAVE + lane(), g.hi - 1u);
      dg[i] = text[o + cyc(n - 1u - (k - o) + (INIT_BYTES - 1u), n)];
    }
  } else {
#pragma unroll
    for (int i = 0; i < RI; i++) dg[i] = kin[min(wbase + i * BZG_WAVE + lane(), g.hi - 1u)];
#pragma unroll
    for (int i = 0; i < RI; i++) dg[i] = (dg[i] >> shift) & 255u;
  }
  uint32_t* mine = cnt + (w * 4u + (lane() & 3u)) * CS;
#pragma unroll
  for (int i = 0; i < RI; i++) {
    const uint32_t k = wbase + i * BZG_WAVE + lane();
    const bool ok = k < g.hi;
    const uint64_t valid = __ballot(ok);
    if (valid) {
      const uint32_t fl = lowest_lane(valid);
      const uint32_t d0 = __builtin_amdgcn_readlane(dg[i], fl);
      const bool same = dg[i] == d0;
      const uint64_t m = __ballot(ok && same);
      if (ok && (!same || lane() == fl)) atomicAdd(&mine[dg[i]], same ? (uint32_t)__popcll(m) : 1u);
    }
  }
  __syncthreads();
  uint32_t d = threadIdx.x;
  uint32_t s = 0;
#pragma unroll
  for (uint32_t q = 0; q < NC; q++) s += cnt[q * CS + d];
  hist[(size_t)g.r.base * 256 + (size_t)d * g.nt + g.t] = s;
}

// Tiles of the scan that follows a histogram pass (its scratch).
__host__ __device__ inline uint32_t hist_scan_states(uint32_t tiles) { return (tiles * 256u + 2047u) / 2048u + 1u; }

// Workgroups over *ntiles tiles of large segments.
template <bool INIT>
__global__ __launch_bounds__(NT) void k_radix_hist(const SegRec* __restrict__ segs, const uint32_t* __restrict__ owner,
                                                   const uint32_t* __restrict__ kin, int shift,
                                                   uint32_t* __restrict__ hist, const uint8_t* __restrict__ text,
                                                   const uint32_t* __restrict__ ntiles, uint32_t cap) {
  const uint32_t n = min(*ntiles, cap);
  for (TileLoop it = tile_loop(n); it.t < it.end; it.t += it.step) {
    radix_hist_tile<INIT>(it.t, segs, owner, kin, shift, hist, text);
    __syncthreads();
  }
}

// One stable LSD pass: (key, row) pairs move.  INIT instantiates the init
// sort's passes; in its first (text != null) rows come from the row index,
// in descending start order, and each key is its row's first INIT_BYTES
// bytes (big-endian, in the high bytes), read sequentially from the text.
template <bool INIT>
__device__ void radix_scatter_tile(uint32_t jt, const SegRec* __restrict__ segs, const uint32_t* __restrict__ owner,
                                   const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                   uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int shift,
                                   const uint32_t* __restrict__ hscan, const uint8_t* __restrict__ text) {
  __shared__ uint32_t cnt[NW][256];
  const uint32_t w = threadIdx.x / BZG_WAVE;
  for (int d = threadIdx.x; d < NW * 256; d += NT) (&cnt[0][0])[d] = 0;
  __syncthreads();
  BigTile g = big_tile(jt, segs, owner);
  const bool from_text = INIT && text != nullptr;
  // this tile's output base for digit threadIdx.x, loaded before the rows
  const size_t col0 = (size_t)g.r.base * 256;
  const uint32_t hs_d = hscan[col0 + (size_t)threadIdx.x * g.nt + g.t], hs_0 = hscan[col0];
  const uint32_t wbase = g.lo + w * (RI * BZG_WAVE);
  // loads of clamped rows, none under a branch, so all are in flight at once
  uint32_t key[RI], val[RI], rk[RI];
  if (from_text) {
    const uint32_t o = g.r.start, n = g.r.len;
    TextWords tw[RI];
#pragma unroll
    for (int i = 0; i < RI; i++) {
      const uint32_t k = min(wbase + i * BZG_WAVE + lane(), g.hi - 1u);
      tw[i] = text_key_load(text, o, n, n - 1u - (k - o));
    }
#pragma unroll
    for (int i = 0; i < RI; i++) {
      const uint32_t k = min(wbase + i * BZG_WAVE + lane(), g.hi - 1u);
      const uint32_t pos = n - 1u - (k - o);
      val[i] = o + pos;
      key[i] = text_key_value(tw[i], text, o, n, pos) & INIT_MASK;
    }
  } else {
#pragma unroll
    for (int i = 0; i < RI; i++) {
      const uint32_t k = min(wbase + i * BZG_WAVE + lane(), g.hi - 1u);
      // streamed once: non-temporal, so the L2 keeps the output runs that
      // neighbouring tiles complete
      key[i] = __builtin_nontemporal_load(&kin[k]);
      val[i] = __builtin_nontemporal_load(&vin[k]);
    }
  }
#pragma unroll
  for (int i = 0; i < RI; i++) {
    const uint32_t k = wbase + i * BZG_WAVE + lane();
    const bool ok = k < g.hi;
    const uint64_t valid = __ballot(ok);
    const uint32_t d = (key[i] >> shift) & 255u;
    rk[i] = 0xFFFFFFFFu;
    if (valid) {
      uint64_t peers = match_digit8(d, valid);
      uint32_t before = cnt[w][d];
      if (ok) rk[i] = before + __popcll(peers & lanemask_lt());
      if (ok && lowest_lane(peers) == lane()) cnt[w][d] = before + __popcll(peers);
    }
  }
  __syncthreads();
  // The tile is staged in LDS in digit order, then every digit's run is
  // written out by consecutive lanes to consecutive addresses.
  __shared__ uint32_t sval[RADIX_TILE], skey[RADIX_TILE];
  __shared__ uint32_t gofs[256];  // output row of a digit's run minus its tile position
  __shared__ uint32_t sh[NW + 1];
  {
    const uint32_t d = threadIdx.x;  // NT == 256: one digit per thread
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < NW; q++) tot += cnt[q][d];
    uint32_t all;
    uint32_t run = block_excl_sum<uint32_t, NT>(tot, sh, &all);
    gofs[d] = g.r.start + hs_d - hs_0 - run;
#pragma unroll
    for (int q = 0; q < NW; q++) {
      uint32_t c = cnt[q][d];
      cnt[q][d] = run;
      run += c;
    }
  }
  __syncthreads();
  // Each stage below reads LDS for all of the thread's items before using
  // any (clamped or unconditional reads), so the reads are in flight
  // together instead of one round trip per item.
  {
    uint32_t base[RI];
#pragma unroll
    for (int i = 0; i < RI; i++) base[i] = cnt[w][(key[i] >> shift) & 255u];
#pragma unroll
    for (int i = 0; i < RI; i++) {
      if (rk[i] != 0xFFFFFFFFu) {
        const uint32_t L = base[i] + rk[i];
        sval[L] = val[i];
        skey[L] = key[i];
      }
    }
  }
  __syncthreads();
  const uint32_t tn = g.hi - g.lo;
  uint32_t kd[RI], vd[RI], go[RI];
#pragma unroll
  for (int i = 0; i < RI; i++) {
    const uint32_t L = min(i * NT + threadIdx.x, tn - 1u);
    kd[i] = skey[L];
    vd[i] = sval[L];
  }
#pragma unroll
  for (int i = 0; i < RI; i++) go[i] = gofs[(kd[i] >> shift) & 255u];
#pragma unroll
  for (int i = 0; i < RI; i++) {
    const uint32_t L = i * NT + threadIdx.x;
    if (L < tn) {
      kout[go[i] + L] = kd[i];
      vout[go[i] + L] = vd[i];
    }
  }
}

template <bool INIT>
__global__ __launch_bounds__(NT) void k_radix_scatter(const SegRec* __restrict__ segs,
                                                      const uint32_t* __restrict__ owner,
                                                      const uint32_t* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                      uint32_t* __restrict__ vout, int shift,
                                                      const uint32_t* __restrict__ hscan,
                                                      const uint8_t* __restrict__ text,
                                                      const uint32_t* __restrict__ ntiles, uint32_t cap) {
  for (TileLoop it = tile_loop(min(*ntiles, cap)); it.t < it.end; it.t += it.step) {
    radix_scatter_tile<INIT>(it.t, segs, owner, kin, vin, kout, vout, shift, hscan, text);
    __syncthreads();
  }
}

// --------------------------------------------------------- new segments

struct AppendCtx {
  SegRec* segs;     // large segments
  uint32_t* head;   // small segments, packed by block: first row + 1 at a segment's first position, else 0
  uint32_t* bcnt;   // packed elements of each block's small segments
  const uint32_t* blk_off;  // block row offsets: block b packs from head[blk_off[b]] on
  uint32_t* owner;  // tile -> large segment index
  RoundCounters* cnt;
  // capacities of segs and owner (every valid input stays below them; an
  // append past one is dropped and flagged)
  uint32_t seg_cap, owner_cap;
  uint32_t* err;
};

// Workgroup-aggregated append of up to `m` groups held by this thread
// (group g = rows [start[g], start[g] + len[g]) of block `blk`, the same
// block for the whole workgroup).  All threads must call it.  Small groups
// are packed into their block's range of the head array (a block's groups
// never hold more elements than it has rows); large groups get a segment
// record and their radix tiles.
template <int M>
__device__ void append_groups(const AppendCtx& a, const uint32_t* gs, const uint32_t* gl, int m, uint32_t blk,
                              uint32_t* wg_base /*LDS[4]*/) {
  uint32_t nseg = 0, nsmall = 0, ntiles = 0, nbig = 0;
  // loops over the M slots with a mask: gs[] and gl[] stay in registers
#pragma unroll
  for (int g = 0; g < M; g++) {
    const uint32_t len = g < m ? gl[g] : 0u;
    const bool big = len > SMALL_MAX;
    nseg += big ? 1u : 0u;
    nsmall += big ? 0u : len;
    ntiles += big ? (len + RADIX_TILE - 1) / RADIX_TILE : 0u;
    nbig += big ? len : 0u;
  }
  // one scan of four packed counts.  Groups appended by a workgroup end in
  // its (at most 4096) rows: segments <= 2048+1, small rows <= 4096+1024,
  // tiles <= 2^21/4096+4 (13 bits each); large rows <= 2^21+4096 (22 bits).
  __shared__ uint64_t sh64[NT / BZG_WAVE + 1];
  const uint64_t packed = (uint64_t)nseg | ((uint64_t)nsmall << 13) | ((uint64_t)ntiles << 26) | ((uint64_t)nbig << 39);
  uint64_t tot;
  const uint64_t ex = block_excl_sum<uint64_t, NT>(packed, sh64, &tot);
  const uint32_t M13 = (1u << 13) - 1u;
  const uint32_t t_seg = (uint32_t)tot & M13, t_small = (uint32_t)(tot >> 13) & M13;
  const uint32_t t_tiles = (uint32_t)(tot >> 26) & M13, t_big = (uint32_t)(tot >> 39) & ((1u << 22) - 1u);
  const uint32_t e_seg = (uint32_t)ex & M13, e_small = (uint32_t)(ex >> 13) & M13, e_tiles = (uint32_t)(ex >> 26) & M13;
  const uint32_t area = a.blk_off[blk], rows = a.blk_off[blk + 1] - area;
  if (threadIdx.x == 0) {
    // neither half of a word carries into the other: tiles and large-segment
    // elements of a round stay below 2^32.  The round's packed-element total
    // is summed from the blocks' counts (k_small_tiles), so the word every
    // workgroup would add to is touched only by those that append a large
    // segment.
    const unsigned long long ss = t_seg ? atomicAdd(&a.cnt->segs_small, (unsigned long long)t_seg) : 0ull;
    const unsigned long long tb =
        t_tiles ? atomicAdd(&a.cnt->tiles_big, (unsigned long long)t_tiles | ((unsigned long long)t_big << 32)) : 0ull;
    wg_base[0] = (uint32_t)ss;
    wg_base[1] = t_small ? atomicAdd(&a.bcnt[blk], t_small) : 0u;
    wg_base[2] = (uint32_t)tb;
  }
  __syncthreads();
  const bool fits = (uint64_t)wg_base[0] + t_seg <= a.seg_cap && (uint64_t)wg_base[1] + t_small <= rows &&
                    (uint64_t)wg_base[2] + t_tiles <= a.owner_cap;
  if (!fits) {
    if (threadIdx.x == 0) atomicOr(a.err, ERR_BOUND);
    m = 0;
  }
  // The workgroup's packed range holds its segments back to back: every
  // position is written (0, then each segment's mark at its start), so a
  // head array needs no clearing before it is appended to.
  if (fits)
    for (uint32_t i = wg_base[1] + threadIdx.x; i < wg_base[1] + t_small; i += NT) a.head[area + i] = 0u;
  __syncthreads();
  uint32_t si = wg_base[0] + e_seg, so = area + wg_base[1] + e_small, st = wg_base[2] + e_tiles;
#pragma unroll
  for (int g = 0; g < M; g++) {
    if (g >= m) break;
    if (gl[g] <= SMALL_MAX) {
      a.head[so] = gs[g] + 1;
      so += gl[g];
    } else {
      SegRec r;
      r.start = gs[g];
      r.len = gl[g];
      r.blk = blk;
      const uint32_t nt = (gl[g] + RADIX_TILE - 1) / RADIX_TILE;
      r.base = st;
      for (uint32_t q = 0; q < nt; q++) a.owner[st + q] = si;
      st += nt;
      a.segs[si] = r;
      si++;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------ naming, large

// Per tile: the last group head (row + 1, 0 = none) among sorted keys.
__device__ void rename_a_tile(uint32_t jt, const SegRec* __restrict__ segs, const uint32_t* __restrict__ owner,
                              const uint32_t* __restrict__ kin, uint32_t* __restrict__ agg) {
  __shared__ uint32_t sh[NW + 1];
  BigTile g = big_tile(jt, segs, owner);
  // every key and its predecessor loaded first (clamped rows, unbranched)
  uint32_t kc[RI], kp[RI];
#pragma unroll
  for (int q = 0; q < RI; q++) {
    const uint32_t k = min(g.lo + q * NT + threadIdx.x, g.hi - 1u);
    kc[q] = kin[k];
    kp[q] = kin[k > g.r.start ? k - 1 : k];
  }
  uint32_t best = 0;
#pragma unroll
  for (int q = 0; q < RI; q++) {
    const uint32_t k = g.lo + q * NT + threadIdx.x;
    if (k < g.hi && (k == g.r.start || kc[q] != kp[q])) best = max(best, k + 1);
  }
  best = wave_max(best);
  if (lane() == 0) sh[threadIdx.x / BZG_WAVE] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int q = 0; q < NW; q++) m = max(m, sh[q]);
    agg[jt] = m;
  }
}

// Persistent workgroups over *ntiles tiles.
__global__ __launch_bounds__(NT) void k_rename_a(const SegRec* __restrict__ segs, const uint32_t* __restrict__ owner,
                                                 const uint32_t* __restrict__ kin, uint32_t* __restrict__ agg,
                                                 const uint32_t* __restrict__ ntiles, uint32_t cap) {
  for (TileLoop it = tile_loop(min(*ntiles, cap)); it.t < it.end; it.t += it.step) {
    rename_a_tile(it.t, segs, owner, kin, agg);
    __syncthreads();
  }
}

// Names the groups of sorted large segments: SA rows in place (vin may be
// SA itself), rank of every row = its group's head row, new segments
// appended.  With rank_all = 0 only rows alone in their group get a rank:
// the others are re-sorted next round, which ranks them, and that round
// compares text rather than ranks (so nothing reads their ranks before).
__device__ void rename_b_tile(uint32_t jt, const SegRec* __restrict__ segs, const uint32_t* __restrict__ owner,
                              const uint32_t* __restrict__ kin, const uint32_t* vin, const uint32_t* __restrict__ agg,
                              const uint32_t* __restrict__ blk_off, uint32_t* SA, uint32_t* __restrict__ rank,
                              uint32_t h_next, int key_is_rank, int rank_all, const AppendCtx& app) {
  __shared__ uint32_t sh[NW + 1];
  __shared__ uint32_t sx[NT];
  __shared__ uint32_t s_carry;
  __shared__ uint32_t wg_base[4];
  BigTile g = big_tile(jt, segs, owner);
  {
    // the group head carried in: the last head in the segment's earlier
    // tiles, i.e. the largest of their per-tile last heads (heads grow with
    // the row)
    uint32_t c = 0;
    for (uint32_t q = threadIdx.x; q < g.t; q += NT) c = max(c, agg[jt - g.t + q]);
    c = wave_max(c);
    if (lane() == 0) sx[threadIdx.x / BZG_WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = max(max(sx[0], sx[1]), max(sx[2], sx[3]));
  }
  const uint32_t bo = blk_off[g.r.blk];
  const uint32_t nblk = blk_off[g.r.blk + 1] - bo;
  const bool keep_blk = h_next < nblk;
  const uint32_t segend = g.r.start + g.r.len;
  // the tile's keys (with the neighbours on both sides, where they are in
  // the segment), loaded coalesced into LDS and read blocked; the rows stay
  // in registers, strided, as the stores at the end take them
  __shared__ uint32_t tk[RADIX_TILE + 2];
  const uint32_t tn = g.hi - g.lo;
  uint32_t rows[RI];  // row g.lo + q * NT + threadIdx.x
  {
    uint32_t a[RI];  // loads first (clamped rows, unbranched), then LDS
#pragma unroll
    for (int q = 0; q < RI; q++) {
      const uint32_t i = min(q * NT + threadIdx.x, tn - 1u);
      // streamed once: non-temporal, so the L2 keeps the rank lines that
      // this kernel's scattered writes land in
      a[q] = __builtin_nontemporal_load(&kin[g.lo + i]);
      rows[q] = __builtin_nontemporal_load(&vin[g.lo + i]);
    }
#pragma unroll
    for (int q = 0; q < RI; q++) {
      const uint32_t i = q * NT + threadIdx.x;
      if (i < tn) tk[i + 1] = a[q];
    }
  }
  if (threadIdx.x == 0) {
    tk[0] = g.lo > g.r.start ? kin[g.lo - 1] : 0u;
    tk[tn + 1] = g.hi < segend ? kin[g.hi] : 0u;
  }
  __syncthreads();
  const uint32_t k0 = g.lo + threadIdx.x * RI;  // blocked: RI consecutive rows per thread
  const uint32_t i0 = threadIdx.x * RI;         // its first position in tk (minus the halo)
  // the thread's keys with one neighbour on each side (t[i + 1] is row
  // k0 + i's key), read from LDS all together; tk holds the tile's keys at
  // 1.. with the keys before and after the tile around them
  uint32_t t[RI + 2];
#pragma unroll
  for (int i = 0; i < RI + 2; i++) t[i] = tk[i0 + i];
  uint32_t lastb = 0;
#pragma unroll
  for (int i = 0; i < RI; i++) {
    const uint32_t k = k0 + i;
    const bool head = (k < g.hi) & ((k == g.r.start) | (t[i + 1] != t[i]));
    lastb = head ? k + 1 : lastb;
  }
  __syncthreads();
  uint32_t incl = block_incl_max<uint32_t, NT>(lastb, sh, 0u);
  sx[threadIdx.x] = incl;
  __syncthreads();
  uint32_t hp = threadIdx.x ? sx[threadIdx.x - 1] : 0u;
  hp = max(hp, s_carry);
  // The rank each row's rotation gets (none = 0xFFFFFFFF) goes to tk (read
  // above by every thread before the scan's barriers) and is stored, with
  // the rows, after the append.
  uint32_t gs[RI / 2 + 1], gl[RI / 2 + 1];
  int m = 0;
#pragma unroll
  for (int i = 0; i < RI; i++) {
    uint32_t k = k0 + i;
    if (k < g.hi) {
      if (k == g.r.start || t[i + 1] != t[i]) hp = k + 1;
      const bool end = (k + 1 == segend) || t[i + 2] != t[i + 1];
      // rank rounds: rows of the segment's first group keep the rank they
      // have (the segment's start)
      const bool same_rank = key_is_rank && hp - 1 == g.r.start;
      tk[i0 + i] = !same_rank && (rank_all || (end && hp == k + 1)) ? hp - 1 : 0xFFFFFFFFu;
      if (end) {
        uint32_t len = k + 1 - (hp - 1);
        // closed group: the segment did not split and every partner lies in
        // it, so its rotations are all equal (already in final order)
        const bool closed = key_is_rank && len == g.r.len && t[i + 1] == g.r.start - bo;
        if (len >= 2 && keep_blk && !closed && m < RI / 2 + 1) {
          gs[m] = hp - 1;
          gl[m] = len;
          m++;
        }
      }
    }
  }
  // the append's reservation (atomics, waited for) before the scattered
  // stores, which it would otherwise wait for; its barriers also order the
  // LDS writes above before the reads below
  append_groups<RI / 2 + 1>(app, gs, gl, m, g.r.blk, wg_base);
  // strided: neighbouring lanes store neighbouring rows
#pragma unroll
  for (int q = 0; q < RI; q++) {
    const uint32_t i = q * NT + threadIdx.x;
    if (i < tn) {
      const uint32_t v = rows[q], r = tk[i];
      if (vin != SA) SA[g.lo + i] = v;
      if (r != 0xFFFFFFFFu) rank[v] = r;
    }
  }
}

__global__ __launch_bounds__(NT) void k_rename_b(const SegRec* __restrict__ segs, const uint32_t* __restrict__ owner,
                                                 const uint32_t* __restrict__ kin, const uint32_t* vin,
                                                 const uint32_t* __restrict__ agg, const uint32_t* __restrict__ blk_off,
                                                 uint32_t* SA, uint32_t* __restrict__ rank,
                                                 uint32_t h_next, int key_is_rank, int rank_all, AppendCtx app,
                                                 const uint32_t* __restrict__ ntiles, uint32_t cap) {
  for (TileLoop it = tile_loop(min(*ntiles, cap)); it.t < it.end; it.t += it.step) {
    rename_b_tile(it.t, segs, owner, kin, vin, agg, blk_off, SA, rank, h_next, key_is_rank, rank_all, app);
    __syncthreads();
  }
}

// ------------------------------------------------------------ gather key2

constexpr uint16_t NO_SEG = 0xFFFFu;

// Exclusive suffix minimum over a workgroup: the minimum of v over the
// threads after this one (hi if none).  sh needs NT/64 slots.
template <int NT_>
__device__ __forceinline__ uint32_t block_excl_suffix_min(uint32_t v, uint32_t* sh, uint32_t hi) {
  constexpr int NWV = NT_ / BZG_WAVE;
  const uint32_t l = lane(), w = threadIdx.x / BZG_WAVE;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < BZG_WAVE; d <<= 1) {
    const uint32_t u = __shfl_down(inc, d, BZG_WAVE);
    if (l + d < BZG_WAVE) inc = min(inc, u);
  }
  if (l == 0) sh[w] = inc;  // the wave's minimum
  __syncthreads();
  uint32_t later = hi;
#pragma unroll
  for (int q = 0; q < NWV; q++) later = q > (int)w ? min(later, sh[q]) : later;
  uint32_t ex = __shfl_down(inc, 1, BZG_WAVE);
  ex = l + 1 < BZG_WAVE ? ex : hi;
  __syncthreads();
  return min(ex, later);
}

// Small tiles.  Block b's small segments are packed from head[blk_off[b]]
// on (bcnt[b] elements); its tiles are the SMALL_T-element windows of that
// range, each taking the segments that start in it.  The tiles of all
// blocks are numbered in block order (tile_pre[b] = the first of block b's,
// tile_pre[nslot] = all), so that neighbouring tiles share a block's text
// and ranks.
struct SmallTile {
  uint32_t blk, lo, avail;  // block, first packed position, packed elements in reach (<= SMALL_CAP)
};
__device__ __forceinline__ SmallTile small_tile_at(uint32_t t, const uint32_t* __restrict__ tile_pre, uint32_t nslot,
                                                   const uint32_t* __restrict__ bcnt,
                                                   const uint32_t* __restrict__ blk_off) {
  // the block whose tiles hold t: tile_pre[b] <= t < tile_pre[b + 1]
  uint32_t lo = 0, hi = nslot;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tile_pre[mid] <= t) lo = mid;
    else hi = mid;
  }
  SmallTile st;
  st.blk = lo;
  const uint32_t k = (t - tile_pre[lo]) * SMALL_T, base = blk_off[lo];
  const uint32_t used = min(bcnt[lo], blk_off[lo + 1] - base);
  st.lo = base + k;
  st.avail = min(used - k, SMALL_CAP);  // >= 1: the tile exists because k < used
  return st;
}

// Loads a small tile's segment map: mark[p] = the segment's first row + 1 at
// each segment's first position, segp[p] = first position of p's segment;
// *s_maxlen gets the longest segment; send (optional) gets each segment's end
// at its first position.  Packed small segments follow each other without
// gaps, so a segment ends where the next one starts (or where the packed rows
// end): one load of the head entries of the tile and of the SMALL_MAX
// positions after it gives every length.
constexpr int PH = SMALL_CAP / NT;  // head entries per thread

// The head entries in a small tile's reach, PH per thread (clamped
// positions: every load is unconditional).
__device__ __forceinline__ void small_tile_heads(const SmallTile& tl, const uint32_t* __restrict__ head,
                                                 uint32_t* hd) {
#pragma unroll
  for (int j = 0; j < PH; j++) hd[j] = head[tl.lo + min(j * NT + threadIdx.x, tl.avail - 1u)];
}

__device__ uint32_t small_tile_map(const SmallTile& tl, const uint32_t* hd, uint32_t* mark, uint16_t* segp,
                                   uint32_t* sh, uint32_t* s_n, uint32_t* s_maxlen, uint16_t* send = nullptr) {
  if (threadIdx.x == 0) {
    *s_n = 0;
    *s_maxlen = 0;
  }
  const uint32_t avail = tl.avail;  // packed rows from the tile's first on, in its reach
#pragma unroll
  for (int j = 0; j < PH; j++) {
    const uint32_t i = j * NT + threadIdx.x;
    mark[i] = i < avail ? hd[j] : 0u;
  }
  __syncthreads();
  constexpr int PER = SMALL_CAP / NT;  // 8 positions per thread, blocked
  const uint32_t p0 = threadIdx.x * PER;
  uint32_t mk[PER];
#pragma unroll
  for (int i = 0; i < PER; i++) mk[i] = mark[p0 + i];
  uint32_t first = avail;  // this thread's first segment start
#pragma unroll
  for (int i = PER - 1; i >= 0; i--) first = mk[i] ? p0 + i : first;
  uint32_t nx = block_excl_suffix_min<NT>(first, sh, avail);  // the next start after the thread's range
  uint32_t en = 0, ml = 0;
#pragma unroll
  for (int i = PER - 1; i >= 0; i--) {
    const uint32_t p = p0 + i;
    if (mk[i]) {
      if (p < SMALL_T) {  // a segment of this tile: it ends at the next start
        en = max(en, nx);
        ml = max(ml, nx - p);
        if (send) send[p] = (uint16_t)nx;
      }
      nx = p;
    }
  }
  // one LDS atomic per wave (same-address atomics serialize)
  en = wave_max(en);
  ml = wave_max(ml);
  if (lane() == 0) {
    atomicMax(s_n, en);
    atomicMax(s_maxlen, ml);
  }
  // only this tile's segment starts stay marked
  uint32_t last = 0;
#pragma unroll
  for (int i = 0; i < PER; i++) {
    if (p0 + i >= SMALL_T) mk[i] = 0;
    last = mk[i] ? p0 + i + 1 : last;
  }
  uint32_t incl = block_incl_max<uint32_t, NT>(last, sh, 0u);
  // exclusive carry via the inclusive value of the previous thread
  __shared__ uint32_t sx[NT];
  sx[threadIdx.x] = incl;
  __syncthreads();
  uint32_t cur = threadIdx.x ? sx[threadIdx.x - 1] : 0u;
#pragma unroll
  for (int i = 0; i < PER; i++) {
    if (mk[i]) cur = p0 + i + 1;
    mark[p0 + i] = mk[i];
    // positions before the tile's first segment belong to a segment of the
    // previous tile
    segp[p0 + i] = cur ? (uint16_t)(cur - 1) : NO_SEG;
  }
  __syncthreads();
  return *s_n;
}

// key2 of every row of every segment: the rank of the rotation h positions
// on, relative to the block start; or (text != null, the first round,
// h = INIT_BYTES) that rotation's first 4 bytes, which order the rows of a
// group (equal in their first h bytes) by their first h + 4.
// key2 of M rows from their partner positions p[i], local to the block at
// bo[i] with bn[i] rows (ONE_BLOCK: all in the block bo[0], bn[0]): the
// partner's rank relative to the block start, or (text != null) its first 4
// bytes.  Every load is issued before any value is used.
template <int M, bool ONE_BLOCK>
__device__ __forceinline__ void gather_keys_impl(uint32_t* p, const uint32_t* bo, const uint32_t* bn,
                                                 const uint8_t* __restrict__ text,
                                                 const uint32_t* __restrict__ rank) {
  if (text) {
    TextWords tw[M];
#pragma unroll
    for (int i = 0; i < M; i++) tw[i] = text_key_load(text, bo[ONE_BLOCK ? 0 : i], bn[ONE_BLOCK ? 0 : i], p[i]);
#pragma unroll
    for (int i = 0; i < M; i++)
      p[i] = text_key_value(tw[i], text, bo[ONE_BLOCK ? 0 : i], bn[ONE_BLOCK ? 0 : i], p[i]);
  } else {
#pragma unroll
    for (int i = 0; i < M; i++) p[i] = rank[bo[ONE_BLOCK ? 0 : i] + p[i]];
#pragma unroll
    for (int i = 0; i < M; i++) p[i] -= bo[ONE_BLOCK ? 0 : i];
  }
}

// A round's sizes from its counter record, clamped to the arrays'
// capacities (an append past a capacity was dropped and flagged, but its
// counts went in).
struct RoundSizes {
  uint32_t nsmall, big_tiles;
};
__device__ __forceinline__ RoundSizes round_sizes(const RoundCounters* c, const uint32_t* tile_pre, uint32_t nslot,
                                                  uint32_t owner_cap) {
  RoundSizes z;
  z.nsmall = tile_pre[nslot];
  z.big_tiles = min(c->big_tiles(), owner_cap);
  return z;
}

// Tiles of each block's packed small segments and their exclusive prefix
// over the blocks (tile_pre, nslot + 1 entries), and the packed elements of
// all blocks (*small_rows).  One workgroup; each thread takes a run of
// consecutive blocks.
constexpr int TS_NT = 1024;
__global__ __launch_bounds__(TS_NT) void k_small_tiles(const uint32_t* __restrict__ bcnt,
                                                      const uint32_t* __restrict__ blk_off, uint32_t nslot,
                                                      uint32_t* __restrict__ tile_pre,
                                                      uint32_t* __restrict__ small_rows) {
  __shared__ uint64_t sh[TS_NT / BZG_WAVE + 1];
  const uint32_t per = (nslot + TS_NT - 1) / TS_NT;
  const uint32_t lo = min(threadIdx.x * per, nslot), hi = min(lo + per, nslot);
  uint64_t acc = 0;  // tiles | elements << 32
  for (uint32_t b = lo; b < hi; b++) {
    const uint32_t c = min(bcnt[b], blk_off[b + 1] - blk_off[b]);
    acc += (uint64_t)((c + SMALL_T - 1) / SMALL_T) | ((uint64_t)c << 32);
  }
  uint64_t tot;
  uint32_t run = (uint32_t)block_excl_sum<uint64_t, TS_NT>(acc, sh, &tot);
  for (uint32_t b = lo; b < hi; b++) {
    tile_pre[b] = run;
    run += (min(bcnt[b], blk_off[b + 1] - blk_off[b]) + SMALL_T - 1) / SMALL_T;
  }
  if (threadIdx.x == 0) {
    tile_pre[nslot] = (uint32_t)tot;
    *small_rows = (uint32_t)(tot >> 32);
  }
}

__device__ void gather_tile(uint32_t jt, uint32_t n_small_tiles, const uint32_t* __restrict__ tile_pre,
                            uint32_t nslot, const uint32_t* __restrict__ bcnt, const SegRec* __restrict__ segs,
                            const uint32_t* __restrict__ head, const uint32_t* __restrict__ owner,
                            const uint32_t* __restrict__ blk_off, const uint32_t* __restrict__ SA,
                            const uint32_t* __restrict__ rank, const uint8_t* __restrict__ text, uint32_t h,
                            uint32_t* __restrict__ key2) {
  __shared__ uint32_t mark[SMALL_CAP];
  __shared__ uint16_t segp[SMALL_CAP];
  __shared__ uint32_t sh[NW + 1];
  __shared__ uint32_t s_n, s_maxlen;
  if (jt < n_small_tiles) {
    const SmallTile tl = small_tile_at(jt, tile_pre, nslot, bcnt, blk_off);
    uint32_t hd[PH];
    small_tile_heads(tl, head, hd);
    uint32_t n = small_tile_map(tl, hd, mark, segp, sh, &s_n, &s_maxlen);
    const uint32_t o = blk_off[tl.blk], nbk = blk_off[tl.blk + 1] - o;
    // rows (from the segment marks), then the rows' SA entries, then the
    // gathers: each stage's loads are issued together, for half the tile at
    // a time (which bounds the registers held across them)
    constexpr int PL = SMALL_CAP / NT / 2;
#pragma unroll 1
    for (int half = 0; half < 2; half++) {
      uint32_t row[PL], kv[PL];
      bool has[PL];
#pragma unroll
      for (int j = 0; j < PL; j++) {
        const uint32_t p = (half * PL + j) * NT + threadIdx.x;
        const uint32_t spv = segp[p];
        const uint32_t mk = mark[spv != NO_SEG ? spv : 0u];
        has[j] = (p < n) & (spv != NO_SEG);
        row[j] = has[j] ? mk - 1u + (p - spv) : o;  // positions without a row read the block's first
      }
#pragma unroll
      for (int j = 0; j < PL; j++) kv[j] = SA[row[j]];
#pragma unroll
      for (int j = 0; j < PL; j++) kv[j] = cyc(kv[j] - o + h, nbk);  // partner position
      gather_keys_impl<PL, true>(kv, &o, &nbk, text, rank);
#pragma unroll
      for (int j = 0; j < PL; j++)
        if (has[j]) key2[row[j]] = kv[j];
    }
  } else {
    BigTile g = big_tile(jt - n_small_tiles, segs, owner);
    const uint32_t o = blk_off[g.r.blk], nbk = blk_off[g.r.blk + 1] - o;
    // all rows of the tile first, then the gathers (independent loads), for
    // half the tile at a time
    constexpr int RH = RI / 2;
#pragma unroll 1
    for (int half = 0; half < 2; half++) {
      uint32_t kv[RH];
#pragma unroll
      for (int q = 0; q < RH; q++) kv[q] = SA[min(g.lo + (half * RH + q) * NT + threadIdx.x, g.hi - 1u)];
#pragma unroll
      for (int q = 0; q < RH; q++) kv[q] = cyc(kv[q] - o + h, nbk);
      gather_keys_impl<RH, true>(kv, &o, &nbk, text, rank);
#pragma unroll
      for (int q = 0; q < RH; q++) {
        const uint32_t k = g.lo + (half * RH + q) * NT + threadIdx.x;
        if (k < g.hi) key2[k] = kv[q];
      }
    }
  }
}

// key2 of this round's segments: persistent workgroups over the small tiles
// (none in the text round, whose small segments gather their own keys) and
// the large segments' tiles.  Workgroup 0 also clears the counter record
// `clr`, the one that the round after the next appends to (nothing reads or
// writes it meanwhile), and the workgroups clear the block counts
// `bcnt_clr`, the ones this round's appends go to (last read by the round
// before).
__global__ __launch_bounds__(NT) void k_gather(const SegRec* __restrict__ segs, const uint32_t* __restrict__ head,
                                               const uint32_t* __restrict__ owner, const RoundCounters* cnt,
                                               const uint32_t* __restrict__ tile_pre,
                                               const uint32_t* __restrict__ bcnt, uint32_t nslot,
                                               RoundCounters* clr, uint32_t* __restrict__ bcnt_clr, int with_small,
                                               uint32_t owner_cap, const uint32_t* __restrict__ blk_off,
                                               const uint32_t* __restrict__ SA, const uint32_t* __restrict__ rank,
                                               const uint8_t* __restrict__ text, uint32_t h,
                                               uint32_t* __restrict__ key2) {
  const RoundSizes z = round_sizes(cnt, tile_pre, nslot, owner_cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clr->segs_small = 0ull;
    clr->tiles_big = 0ull;
  }
  for (uint32_t b = blockIdx.x * NT + threadIdx.x; b < nslot; b += gridDim.x * NT) bcnt_clr[b] = 0u;
  const uint32_t nsmall = with_small ? z.nsmall : 0u;
  for (TileLoop it = tile_loop(nsmall + z.big_tiles); it.t < it.end; it.t += it.step) {
    gather_tile(it.t, nsmall, tile_pre, nslot, bcnt, segs, head, owner, blk_off, SA, rank, text, h, key2);
    __syncthreads();
  }
}

// --------------------------------------------------- small segments, LDS

// Sorts packed small segments in LDS, names their groups, ranks their rows
// and appends the groups that stay unresolved.  Rank rounds sort on
// (segment position << 21 | key2) in 4 passes; the text round (text_mode,
// 32-bit keys) sorts on key2 and then the segment position, 6 passes, and
// leaves equal-rotation groups to the next round.
// A tile is ordered by counting instead of radix passes when the counting
// costs its slowest wave at most this many steps per radix pass the tile
// would otherwise run (a counting step of 64 rows and a radix pass over 64
// rows cost about this much in issued instructions, measured as counters).
constexpr uint32_t COUNT_STEPS_PER_PASS = 48;  // (the built-in choice; a context may set another)

__device__ void small_sort_tile(const SmallTile& tl, const uint32_t* hd, uint32_t jt_next, SmallTile& tl_next,
                                uint32_t* hd_next, const uint32_t* __restrict__ tile_pre, uint32_t nslot,
                                const uint32_t* __restrict__ bcnt, const uint32_t* __restrict__ head,
                                const uint32_t* __restrict__ blk_off,
                                const uint32_t* __restrict__ key2, uint32_t* __restrict__ SA,
                                uint32_t* __restrict__ rank, uint32_t h, uint32_t h_next,
                                const uint8_t* __restrict__ text, const AppendCtx& app, uint32_t count_steps) {
  const bool text_mode = text != nullptr;
  __shared__ uint32_t mark[SMALL_CAP];
  __shared__ uint32_t sval[SMALL_CAP];
  __shared__ uint16_t segp[SMALL_CAP];
  __shared__ uint32_t skey[SMALL_CAP];
  __shared__ uint16_t sseg[SMALL_CAP];  // segment ends (counting) or each key's segment position (radix)
  __shared__ uint32_t scnt[NW][256];
  __shared__ uint32_t sh[NW + 1];
  __shared__ uint32_t sx[NT];
  __shared__ uint32_t s_n, s_maxlen, s_cost;
  __shared__ uint32_t wg_base[4];
  if (threadIdx.x == 0) s_cost = 0;
  const uint32_t n = small_tile_map(tl, hd, mark, segp, sh, &s_n, &s_maxlen, sseg);
  // the tile's block (one per tile)
  const uint32_t bo = blk_off[tl.blk], nbk = blk_off[tl.blk + 1] - bo;
  constexpr int PI = SMALL_CAP / NT;  // 8
  const int npass_radix = text_mode ? 6 : 4;
  // Counting (below) ranks each row among its segment's rows in as many
  // steps as the longest segment among the wave's 64 positions; the tile is
  // counted when its slowest wave's steps cost less than the radix passes.
  // Counted tiles keep the segment ends in sseg.
  {
    uint32_t steps = 0;
#pragma unroll
    for (int j = 0; j < PI; j++) {
      const uint32_t p = j * NT + threadIdx.x;
      const uint32_t spv = p < n ? segp[p] : NO_SEG;
      const uint32_t len = spv != NO_SEG ? (uint32_t)sseg[spv] - spv : 0u;
      steps += wave_max(len);
    }
    if (lane() == 0) atomicMax(&s_cost, steps);
  }
  __syncthreads();
  const bool counting = s_cost <= count_steps * (uint32_t)npass_radix;
  // load (segment start << 21 | key2, SA value).  Positions before the
  // first segment take key 0 and stay in front (no segment starts at 0 then);
  // positions past the last take the largest key and stay behind.
  {
    // rows from the segment marks, then their key2 and SA entries (independent
    // loads, issued together); positions without a row load the block's first
    // row, so that no load sits under a branch and each stage's loads are all
    // in flight together
    constexpr int PL = SMALL_CAP / NT;
    uint32_t sp[PL], kk[PL], k2[PL], vv[PL];
#pragma unroll
    for (int j = 0; j < PL; j++) {
      const uint32_t p = j * NT + threadIdx.x;
      sp[j] = p < n ? segp[p] : NO_SEG;
      const uint32_t mk = mark[sp[j] != NO_SEG ? sp[j] : 0u];
      kk[j] = sp[j] != NO_SEG ? mk - 1u + (p - sp[j]) : bo;
    }
#pragma unroll
    for (int j = 0; j < PL; j++) {
      if (!text) k2[j] = key2[kk[j]];
      vv[j] = SA[kk[j]];
    }
    if (text) {
      // the text round gathers its own keys: the first 4 bytes of the
      // rotation h positions on (no k_gather pass for small segments)
#pragma unroll
      for (int j = 0; j < PL; j++) k2[j] = cyc(vv[j] - bo + h, nbk);
      gather_keys_impl<PL, true>(k2, &bo, &nbk, text, nullptr);
    }
    // (selects, not branches: a load used only under a branch would be
    // moved into it and waited for there)
#pragma unroll
    for (int j = 0; j < PL; j++) {
      const uint32_t p = j * NT + threadIdx.x;
      const bool has = sp[j] != NO_SEG, front = !has && p < n;  // front: before the tile's first segment
      const uint32_t kr = text_mode ? k2[j] : (sp[j] << 21) | k2[j];
      skey[p] = has ? kr : front ? 0u : 0xFFFFFFFFu;
      sval[p] = has ? vv[j] : 0u;
      if (!counting) sseg[p] = (uint16_t)(has ? sp[j] : front ? 0u : 0xFFFFu);
    }
  }
  __syncthreads();
  // stable LSD radix sort of the tile in LDS; wave w owns positions
  // [w*1024, (w+1)*1024), item i of lane l is position w*1024 + i*64 + l
  const uint32_t w = threadIdx.x / BZG_WAVE;
  // Counting: for every row, the rows of its segment that precede it
  // (smaller key, or equal key further up); keys compare equal inside a
  // segment exactly when key2 does.
  if (counting) {
    uint32_t dst[PI], kv[PI], vv[PI];
#pragma unroll
    for (int j = 0; j < PI; j++) {
      const uint32_t p = j * NT + threadIdx.x;
      const uint32_t spv = p < n ? segp[p] : NO_SEG;
      const bool has = spv != NO_SEG;
      const uint32_t sp = has ? spv : 0u;
      const uint32_t len = has ? (uint32_t)sseg[sp] - sp : 0u, d = p - sp;
      const uint32_t me = skey[p];
      // the wave steps through the longest segment among its positions
      const uint32_t wl = wave_max(len);
      uint32_t r = 0;
      // (bitwise, not short-circuit, tests: a load used only under a branch
      // would be moved into it and waited for there, one LDS round trip per
      // step)
#pragma unroll 8
      for (uint32_t i = 0; i < wl; i++) {
        const uint32_t o = skey[min(sp + i, SMALL_CAP - 1u)];
        r += (uint32_t)(i < len) & ((uint32_t)(o < me) | ((uint32_t)(o == me) & (uint32_t)(i < d)));
      }
      dst[j] = has ? sp + r : 0xFFFFFFFFu;
      kv[j] = me;
      vv[j] = sval[p];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PI; j++)
      if (dst[j] != 0xFFFFFFFFu) {
        skey[dst[j]] = kv[j];
        sval[dst[j]] = vv[j];
      }
    __syncthreads();
  }
  const int npass = counting ? 0 : npass_radix;
  // the passes sort positions [0, 4 * 64 * R) only, R items per lane: the
  // positions from n on hold the largest key and stay behind anyway
  const int R = (int)((n + NW * BZG_WAVE - 1) / (NW * BZG_WAVE));
  for (int pass = 0; pass < npass; pass++) {
    const int shift = (pass & 3) * 8;
    const bool by_seg = pass >= 4;  // text round: the segment position last
    for (int d = threadIdx.x; d < NW * 256; d += NT) (&scnt[0][0])[d] = 0;
    __syncthreads();
    uint32_t key[PI], val[PI], rk[PI], sg[PI];
#pragma unroll
    for (int i = 0; i < PI; i++) {
      if (i >= R) break;
      uint32_t p = (w * R + i) * BZG_WAVE + lane();
      key[i] = skey[p];
      val[i] = sval[p];
      sg[i] = sseg[p];
      uint32_t d = ((by_seg ? sg[i] : key[i]) >> shift) & 255u;
      uint64_t peers = match_digit8(d, ~0ull);
      uint32_t before = scnt[w][d];
      rk[i] = before + __popcll(peers & lanemask_lt());
      if (lowest_lane(peers) == lane()) scnt[w][d] = before + __popcll(peers);
    }
    __syncthreads();
    {
      uint32_t d = threadIdx.x;
      uint32_t tot = 0;
#pragma unroll
      for (int q = 0; q < NW; q++) tot += scnt[q][d];
      uint32_t all;
      uint32_t run = block_excl_sum<uint32_t, NT>(tot, sh, &all);
#pragma unroll
      for (int q = 0; q < NW; q++) {
        uint32_t c = scnt[q][d];
        scnt[q][d] = run;
        run += c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PI; i++) {
      if (i >= R) break;
      uint32_t d = ((by_seg ? sg[i] : key[i]) >> shift) & 255u;
      uint32_t pos = scnt[w][d] + rk[i];
      skey[pos] = key[i];
      sval[pos] = val[i];
      sseg[pos] = (uint16_t)sg[i];
    }
    __syncthreads();
  }
  // the next tile's head entries, loaded now: before this tile's scattered
  // stores, so that waiting for them later does not wait for the stores
  // (one memory counter covers loads and stores, in issue order)
  if (jt_next != 0xFFFFFFFFu) {
    tl_next = small_tile_at(jt_next, tile_pre, nslot, bcnt, blk_off);
    small_tile_heads(tl_next, head, hd_next);
  }
  // naming: blocked, PI consecutive positions per thread.  The thread's
  // keys (with one neighbour on each side), segment starts and rows are read
  // from LDS first, all together (clamped positions).
  const uint32_t p0 = threadIdx.x * PI;
  uint32_t sk[PI + 2], sg[PI], sv[PI];
#pragma unroll
  for (int i = 0; i < PI + 2; i++) sk[i] = skey[min(max(p0 + i, 1u) - 1u, SMALL_CAP - 1u)];
#pragma unroll
  for (int i = 0; i < PI; i++) {
    sg[i] = segp[p0 + i];
    sv[i] = sval[p0 + i];
  }
  // each position's segment: its first row (the mark at its first
  // position) and whether the segment ends there
  uint32_t rs[PI];
#pragma unroll
  for (int i = 0; i < PI; i++) rs[i] = mark[sg[i] != NO_SEG ? sg[i] : 0u] - 1u;
  const uint32_t sg_next = segp[min(p0 + PI, SMALL_CAP - 1u)];
  uint32_t lastb = 0;
#pragma unroll
  for (int i = 0; i < PI; i++) {
    const uint32_t p = p0 + i;
    const bool head = (p < n) & (sg[i] != NO_SEG) & ((p == sg[i]) | (sk[i + 1] != sk[i]));
    lastb = head ? p + 1 : lastb;
  }
  uint32_t incl = block_incl_max<uint32_t, NT>(lastb, sh, 0u);
  sx[threadIdx.x] = incl;
  __syncthreads();
  uint32_t hp = threadIdx.x ? sx[threadIdx.x - 1] : 0u;
  // Each position's SA row and the rank its rotation gets go to LDS (skey
  // and mark, read above by every thread before the barriers of the scan),
  // none = 0xFFFFFFFF, and are stored after the append.
  uint32_t gs[PI / 2 + 1], gl[PI / 2 + 1];
  int m = 0;
#pragma unroll
  for (int i = 0; i < PI; i++) {
    uint32_t p = p0 + i;
    skey[p] = 0xFFFFFFFFu;
    mark[p] = 0xFFFFFFFFu;
    if (p >= n) continue;
    uint32_t sp = sg[i];
    if (sp == NO_SEG) continue;
    if (p == sp || sk[i + 1] != sk[i]) hp = p + 1;
    const uint32_t headk = rs[i] + (hp - 1 - sp);
    skey[p] = rs[i] + (p - sp);
    // rank rounds: rows of the segment's first group keep the rank they have
    // (the segment's start), so only the other groups' rows are written
    if (text_mode || hp - 1 != sp) mark[p] = headk;
    const bool seg_end = (p + 1 == n) || (i + 1 < PI ? sg[i + 1] : sg_next) != sp;
    const bool end = seg_end || sk[i + 2] != sk[i + 1];
    if (end) {
      uint32_t len = p + 1 - (hp - 1);
      // closed group (see k_rename_b): equal rotations, final
      const bool closed = !text_mode && seg_end && hp - 1 == sp && (sk[i + 1] & ((1u << 21) - 1u)) == rs[i] - bo;
      if (len >= 2 && h_next < nbk && !closed) {
#pragma unroll
        for (int q = 0; q < PI / 2 + 1; q++)  // register-resident append
          if (q == m) {
            gs[q] = headk;
            gl[q] = len;
          }
        m++;
      }
    }
  }
  // the append's reservation (atomics, waited for) before the scattered
  // stores below, which it would otherwise wait for; its barriers also
  // order the LDS writes above before the reads below
  append_groups<PI / 2 + 1>(app, gs, gl, m, tl.blk, wg_base);
  // strided: neighbouring lanes store neighbouring rows of a segment
#pragma unroll
  for (int j = 0; j < PI; j++) {
    const uint32_t p = j * NT + threadIdx.x;
    const uint32_t k = skey[p], r = mark[p], v = sval[p];
    if (k != 0xFFFFFFFFu) SA[k] = v;
    if (r != 0xFFFFFFFFu) rank[v] = r;
  }
}

__global__ __launch_bounds__(NT, 4) void k_small_sort(const uint32_t* __restrict__ head,
                                                   const uint32_t* __restrict__ tile_pre,
                                                   const uint32_t* __restrict__ bcnt, uint32_t nslot,
                                                   const uint32_t* __restrict__ blk_off,
                                                   const uint32_t* __restrict__ key2, uint32_t* __restrict__ SA,
                                                   uint32_t* __restrict__ rank, uint32_t h, uint32_t h_next,
                                                   const uint8_t* __restrict__ text, AppendCtx app,
                                                   uint32_t count_steps) {
  const uint32_t nsmall = tile_pre[nslot];
  TileLoop it = tile_loop(nsmall);
  if (it.t >= it.end) return;
  // each tile's head entries are loaded by the tile before it
  SmallTile tl = small_tile_at(it.t, tile_pre, nslot, bcnt, blk_off);
  uint32_t hd[PH];
  small_tile_heads(tl, head, hd);
  for (; it.t < it.end; it.t += it.step) {
    const uint32_t tn = it.t + it.step < it.end ? it.t + it.step : 0xFFFFFFFFu;
    SmallTile tl_next = tl;
    uint32_t hd_next[PH];
    small_sort_tile(tl, hd, tn, tl_next, hd_next, tile_pre, nslot, bcnt, head, blk_off, key2, SA, rank, h, h_next,
                    text, app, count_steps);
    __syncthreads();
    tl = tl_next;
#pragma unroll
    for (int j = 0; j < PH; j++) hd[j] = hd_next[j];
  }
}

// ------------------------------------------------------------- final BWT

// L[k] = byte before rotation SA[k]; primary[b] = row of rotation 0; the
// optional local SA.  Each thread takes OUT_ROWS consecutive rows (one block
// search, then the block boundary is followed), L is stored a dword at a
// time.
constexpr uint32_t OUT_ROWS = 16;

__device__ __forceinline__ void bwt_out_rows(uint32_t k0, const uint8_t* __restrict__ text,
                                             const uint32_t* __restrict__ off, uint32_t nb, uint32_t N,
                                             const uint32_t* __restrict__ SA, uint8_t* __restrict__ L,
                                             uint32_t* __restrict__ primary, uint32_t* __restrict__ sa_local) {
  if (k0 >= N) return;
  const uint32_t cnt = min(OUT_ROWS, N - k0);
  uint32_t b = find_block(off, nb, k0);
  uint32_t o = off[b], e = off[b + 1];
  uint32_t p[OUT_ROWS];
#pragma unroll
  for (uint32_t i = 0; i < OUT_ROWS; i++) p[i] = i < cnt ? SA[k0 + i] : 0u;
  // text index of every row's last-column byte first, then the gathers
  uint32_t src[OUT_ROWS];
#pragma unroll
  for (uint32_t i = 0; i < OUT_ROWS; i++) {
    src[i] = 0;
    if (i < cnt) {
      const uint32_t k = k0 + i;
      while (k >= e) {  // next block (empty ones are stepped over)
        b++;
        o = e;
        e = off[b + 1];
      }
      const uint32_t q = p[i];
      src[i] = q == o ? e - 1 : q - 1;
      if (q == o) primary[b] = k - o;
      if (sa_local) sa_local[k] = q - o;
    }
  }
  // every gather issued before any is used (rows past cnt re-read row 0's)
  uint32_t t[OUT_ROWS];
#pragma unroll
  for (uint32_t i = 0; i < OUT_ROWS; i++) t[i] = text[i < cnt ? src[i] : src[0]];
  uint32_t w[OUT_ROWS / 4] = {0, 0, 0, 0};
#pragma unroll
  for (uint32_t i = 0; i < OUT_ROWS; i++) w[i >> 2] |= t[i] << (8 * (i & 3));
  if (cnt == OUT_ROWS && ((uintptr_t)(L + k0) & 15u) == 0) {
    *(uint4*)(L + k0) = make_uint4(w[0], w[1], w[2], w[3]);
  } else {
    for (uint32_t i = 0; i < cnt; i++) L[k0 + i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
  }
}

// Persistent workgroups over the *n_rows rows, NT * OUT_ROWS per tile.
__global__ __launch_bounds__(NT) void k_bwt_out(const uint8_t* __restrict__ text, const uint32_t* __restrict__ off,
                                                uint32_t nb, const uint32_t* __restrict__ n_rows, uint32_t cap,
                                                const uint32_t* __restrict__ SA, uint8_t* __restrict__ L,
                                                uint32_t* __restrict__ primary, uint32_t* __restrict__ sa_local) {
  const uint32_t N = min(*n_rows, cap);
  for (TileLoop it = tile_loop((N + NT * OUT_ROWS - 1) / (NT * OUT_ROWS)); it.t < it.end; it.t += it.step)
    bwt_out_rows((it.t * NT + threadIdx.x) * OUT_ROWS, text, off, nb, N, SA, L, primary, sa_local);
}

// ------------------------------------------------------------- host side

static BwtSizes bwt_sizes(uint32_t N, uint32_t nb) {
  BwtSizes z;
  z.seg_cap = N / 2 + nb + 16;
  z.head_cap = N + 16;  // block b packs its small segments from its first row on
  z.owner_cap = N / RADIX_TILE + N / (SMALL_MAX + 1) + nb + 16;
  z.hist_cap = (size_t)z.owner_cap * 256 + 16;
  z.state_cap = hist_scan_states((uint32_t)z.owner_cap) + 16;
  return z;
}

size_t bwt_workspace_bytes(uint32_t N, uint32_t nb) {
  BwtSizes z = bwt_sizes(N, nb);
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  for (int i = 0; i < 5; i++) add((size_t)N * 4 + 64);  // SA rank key tmpK tmpV
  add(z.hist_cap * 4);
  add(z.state_cap * 8);
  add(z.owner_cap * 4);  // agg
  for (int i = 0; i < 2; i++) {
    add(z.seg_cap * sizeof(SegRec));
    add(z.owner_cap * 4);
  }
  add(z.head_cap * 4 * 2);
  for (int i = 0; i < 3; i++) add(((size_t)nb + 1) * 4);  // bcnt[2], tile_pre
  add(3 * sizeof(RoundCounters));
  return b + 4096;
}

bool bwt_carve(void* ws, size_t ws_bytes, uint32_t N, uint32_t nb, BwtWork& w) {
  const BwtSizes z = bwt_sizes(N, nb);
  Bump bump;
  bump.base = (char*)ws;
  bump.cap = ws_bytes;
  w.z = z;
  w.SA = bump.take<uint32_t>(N + 16);
  w.rank = bump.take<uint32_t>(N + 16);
  w.key = bump.take<uint32_t>(N + 16);
  w.tmpK = bump.take<uint32_t>(N + 16);
  w.tmpV = bump.take<uint32_t>(N + 16);
  w.hist = bump.take<uint32_t>(z.hist_cap);
  w.state = bump.take<unsigned long long>(z.state_cap);
  w.agg = bump.take<uint32_t>(z.owner_cap);
  for (int i = 0; i < 2; i++) {
    w.segs[i] = bump.take<SegRec>(z.seg_cap);
    w.owner[i] = bump.take<uint32_t>(z.owner_cap);
  }
  w.head[0] = bump.take<uint32_t>(z.head_cap);
  w.head[1] = bump.take<uint32_t>(z.head_cap);
  w.bcnt[0] = bump.take<uint32_t>((size_t)nb + 1);
  w.bcnt[1] = bump.take<uint32_t>((size_t)nb + 1);
  w.tile_pre = bump.take<uint32_t>((size_t)nb + 1);
  w.nslot = nb;
  w.cnt = bump.take<RoundCounters>(3);
  return bump.used <= ws_bytes;
}

// Doubling rounds after the first sort, while the ordered prefix P is
// shorter than the longest block: P = INIT_BYTES after the init sort,
// INIT_BYTES + 4 after the first round (text), then doubling (groups in
// blocks of at most P rows are then finished).
int bwt_rounds(uint32_t max_len) {
  int r = 0;
  for (uint64_t P = INIT_BYTES; P < max_len; P = r ? 2 * P : P + 4, r++) {
  }
  return r;
}

static hipError_t radix_passes(BwtWork& w, uint32_t cap, const uint32_t* ntiles, const uint32_t* nrows,
                               const SegRec* segs, const uint32_t* owner, int passes, uint32_t* err, uint32_t** kin,
                               uint32_t** vin, hipStream_t st) {
  // round passes: tile counts are device-side and usually far below their
  // bound, so the workgroups are persistent, as many as are resident
  const uint32_t gh = resident_grid((const void*)k_radix_hist<false>, NT);
  const uint32_t gs = resident_grid((const void*)k_radix_scatter<false>, NT);
  const uint32_t gq = std::min(resident_grid((const void*)k_radix_hist<false>, NT),
                               persist_grid(scan_dev_tiles((uint64_t)cap * 256), ONE_TILE_EACH));
  uint32_t *ka = w.key, *va = w.SA, *kb = w.tmpK, *vb = w.tmpV;
  for (int p = 0; p < passes; p++) {
    {
      ProfScope ps("radix_hist", st, 0, nrows, 4.0);  // read the key
      hipLaunchKernelGGL(k_radix_hist<false>, dim3(gh), dim3(NT), 0, st, segs, owner, ka, 8 * p, w.hist, nullptr,
                         ntiles, cap);
    }
    {
      ProfScope ps("sort_scan", st, 0, ntiles, 8.0 * 256);
      hipError_t e = scan_lb_u32(w.hist, ntiles, cap, 256, w.state, err, gq, st);
      if (e != hipSuccess) return e;
    }
    ProfScope ps("radix_scatter", st, 0, nrows, 16.0);  // read and write key and value
    hipLaunchKernelGGL(k_radix_scatter<false>, dim3(gs), dim3(NT), 0, st, segs, owner, ka, va, kb, vb, 8 * p,
                       w.hist, nullptr, ntiles, cap);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  *kin = ka;
  *vin = va;
  return hipGetLastError();
}

// Sorts the rotations of every block of `text` (block b = rows
// [d_off[b], d_off[b+1]), possibly empty, at most bd.max_len each; d_off[nb]
// = the row count, at most bd.rows).  The first segments (one per block,
// w.segs[0]) and their tile owners (w.owner[0], *init_tiles of them) are set
// by the caller.  Every round of the fixed schedule is enqueued; rounds with
// nothing left to sort find zero counts and end at once.  SA rows end in
// w.SA.
hipError_t bwt_sort(BwtWork& w, const uint8_t* text, const uint32_t* d_off, const uint32_t* init_tiles,
                    const BwtBounds& bd, uint32_t* err, int* rounds, hipStream_t st) {
  const BwtSizes& z = w.z;
  // round kernels: persistent, as many workgroups as are resident
  const uint32_t Gg = resident_grid((const void*)k_gather, NT);
  const uint32_t Gs = resident_grid((const void*)k_small_sort, NT);
  const uint32_t Ga = resident_grid((const void*)k_rename_a, NT);
  const uint32_t Gb = resident_grid((const void*)k_rename_b, NT);
  const uint32_t count_steps = g_tune && g_tune->count_steps ? g_tune->count_steps : COUNT_STEPS_PER_PASS;
  hipError_t e;
#define BZG_TRY(x)                  \
  do {                              \
    e = (x);                        \
    if (e != hipSuccess) return e;  \
  } while (0)
  // the counter records and the block counts of the first list start at
  // zero (the second list's are cleared by the first round); the head arrays
  // need no clearing (each append writes its whole range)
  BZG_TRY(fill32((uint32_t*)w.cnt, 3 * sizeof(RoundCounters) / 4, 0u, st));
  BZG_TRY(fill32(w.bcnt[1], w.nslot, 0u, st));
  const uint32_t* rows = d_off + bd.nslot;  // the row count
  const uint32_t icap = std::min<uint32_t>(bd.init_tiles, (uint32_t)z.owner_cap);
  const uint32_t Gi = persist_grid(icap, ONE_TILE_EACH);  // first sort: one tile per workgroup
  const uint32_t Gsi = persist_grid(scan_dev_tiles((uint64_t)icap * 256), ONE_TILE_EACH);
  // init: INIT_BYTES LSD passes on the first bytes of every rotation (the
  // last pass writes w.key / w.SA)
  {
    uint32_t* kout[INIT_BYTES];
    uint32_t* vout[INIT_BYTES];
    for (int p = 0; p < (int)INIT_BYTES; p++) {
      const bool last_parity = ((int)INIT_BYTES - 1 - p) % 2 == 0;
      kout[p] = last_parity ? w.key : w.tmpK;
      vout[p] = last_parity ? w.SA : w.tmpV;
    }
    for (int p = 0; p < (int)INIT_BYTES; p++) {
      const uint32_t* ka = p ? kout[p - 1] : nullptr;
      const uint32_t* va = p ? vout[p - 1] : nullptr;
      const int shift = 8 * (p + 4 - (int)INIT_BYTES);
      {
        ProfScope ps("init_hist", st, 0, rows, p ? 4.0 : 1.0);  // key in (pass 0: one text byte)
        hipLaunchKernelGGL(k_radix_hist<true>, dim3(Gi), dim3(NT), 0, st, w.segs[0], w.owner[0], ka, shift, w.hist,
                           p ? nullptr : text, init_tiles, icap);
      }
      {
        ProfScope ps("sort_scan", st, 0, init_tiles, 8.0 * 256);
        BZG_TRY(scan_lb_u32(w.hist, init_tiles, icap, 256, w.state, err, Gsi, st));
      }
      // key and row in and out (pass 0: one text byte in per row)
      ProfScope ps("init_scatter", st, 0, rows, p ? 16.0 : 9.0);
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3(Gi), dim3(NT), 0, st, w.segs[0], w.owner[0], ka, va, kout[p],
                         vout[p], shift, w.hist, p ? nullptr : text, init_tiles, icap);
    }
  }
  const uint32_t ocap = (uint32_t)z.owner_cap, nslot = std::min(bd.nslot, w.nslot);
  {
    AppendCtx app{w.segs[1], w.head[1], w.bcnt[1], d_off, w.owner[1], &w.cnt[1], (uint32_t)z.seg_cap, ocap, err};
    {
      ProfScope ps("rename_a", st, 0, rows, 4.0);
      hipLaunchKernelGGL(k_rename_a, dim3(Gi), dim3(NT), 0, st, w.segs[0], w.owner[0], w.key, w.agg, init_tiles,
                         icap);
    }
    ProfScope ps("rename_b", st, 0, rows, 12.0);  // key and row in, rank out
    // only rows alone in their group are ranked here: round 0 compares text
    hipLaunchKernelGGL(k_rename_b, dim3(Gi), dim3(NT), 0, st, w.segs[0], w.owner[0], w.key, w.SA, w.agg, d_off, w.SA,
                       w.rank, INIT_BYTES, 0, 0, app, init_tiles, icap);
  }
  BZG_TRY(hipGetLastError());
  int bits = 1;
  while ((1u << bits) < bd.max_len) bits++;
  const int rank_passes = (bits + 7) / 8;
  const int R = bwt_rounds(bd.max_len);
  int cur = 1;  // segment lists and head arrays: double-buffered
  int cc = 1;   // counter records: three, so a round clears the one it does not touch
  uint32_t P = INIT_BYTES;  // the ordered prefix
  for (int r = 0; r < R; r++) {
    const int nxt = cur ^ 1, cn = (cc + 1) % 3, cz = (cc + 2) % 3;
    const bool text_round = r == 0;
    // partners h rows on; after the round rotations are ordered by Pn bytes
    const uint32_t h = P, Pn = text_round ? P + 4 : 2 * P;
    P = Pn;
    const uint32_t* big_tiles = (const uint32_t*)&w.cnt[cc].tiles_big;         // low word
    const uint32_t* small_rows = (const uint32_t*)&w.cnt[cc].segs_small + 1;   // high word
    const uint32_t* big_rows = (const uint32_t*)&w.cnt[cc].tiles_big + 1;      // high word
    {
      ProfScope ps("sort_scan", st, 0.0);
      hipLaunchKernelGGL(k_small_tiles, dim3(1), dim3(TS_NT), 0, st, w.bcnt[cur], d_off, nslot, w.tile_pre,
                         (uint32_t*)small_rows);
    }
    {
      // row, partner rank, key2
      ProfScope ps("gather", st, 0, big_rows, 12.0, text_round ? nullptr : small_rows, 12.0);
      // the text round's small segments gather their keys in k_small_sort
      hipLaunchKernelGGL(k_gather, dim3(Gg), dim3(NT), 0, st, w.segs[cur], w.head[cur], w.owner[cur], &w.cnt[cc],
                         w.tile_pre, w.bcnt[cur], nslot, &w.cnt[cz], w.bcnt[nxt], text_round ? 0 : 1, ocap, d_off,
                         w.SA, w.rank, text_round ? text : nullptr, h, w.key);
    }
    AppendCtx app2{w.segs[nxt], w.head[nxt], w.bcnt[nxt], d_off, w.owner[nxt], &w.cnt[cn], (uint32_t)z.seg_cap,
                   ocap, err};
    {
      ProfScope ps("small_sort", st, 0, small_rows, 16.0);  // key2 and row in, row and rank out
      hipLaunchKernelGGL(k_small_sort, dim3(Gs), dim3(NT), 0, st, w.head[cur], w.tile_pre, w.bcnt[cur], nslot,
                         d_off, w.key, w.SA, w.rank, h, Pn, text_round ? text : nullptr, app2, count_steps);
    }
    uint32_t *kin, *vin;
    BZG_TRY(radix_passes(w, ocap, big_tiles, big_rows, w.segs[cur], w.owner[cur], text_round ? 4 : rank_passes,
                         err, &kin, &vin, st));
    {
      ProfScope ps("rename_a", st, 0, big_rows, 4.0);
      hipLaunchKernelGGL(k_rename_a, dim3(Ga), dim3(NT), 0, st, w.segs[cur], w.owner[cur], kin, w.agg, big_tiles,
                         ocap);
    }
    ProfScope ps("rename_b", st, 0, big_rows, 16.0);
    hipLaunchKernelGGL(k_rename_b, dim3(Gb), dim3(NT), 0, st, w.segs[cur], w.owner[cur], kin, vin, w.agg, d_off, w.SA,
                       w.rank, Pn, text_round ? 0 : 1, 1, app2, big_tiles, ocap);
    BZG_TRY(hipGetLastError());
    cur = nxt;
    cc = cn;
  }
  if (rounds) *rounds = R;
  return hipGetLastError();
#undef BZG_TRY
}

void bwt_warm_grids() {
  (void)resident_grid((const void*)k_gather, NT);
  (void)resident_grid((const void*)k_small_sort, NT);
  (void)resident_grid((const void*)k_rename_a, NT);
  (void)resident_grid((const void*)k_rename_b, NT);
  (void)resident_grid((const void*)k_radix_hist<false>, NT);
  (void)resident_grid((const void*)k_radix_scatter<false>, NT);
}

hipError_t bwt_output(const uint8_t* text, const uint32_t* d_off, uint32_t nb, const uint32_t* n_rows, uint32_t cap,
                      const uint32_t* SA, uint8_t* L, uint32_t* primary, uint32_t* sa_local, hipStream_t st) {
  ProfScope ps("bwt_out", st, 0, n_rows, 6.0);  // row in, byte gathered, byte out
  const uint32_t g = persist_grid(((uint64_t)cap + NT * OUT_ROWS - 1) / (NT * OUT_ROWS), ONE_TILE_EACH);
  hipLaunchKernelGGL(k_bwt_out, dim3(g), dim3(NT), 0, st, text, d_off, nb, n_rows, cap, SA, L, primary, sa_local);
  return hipGetLastError();
}

}  // namespace bzg
