// Block CRC and RLE1 (bzip2's first run-length stage), data-parallel.
//
// RLE1 follows the four-step pattern of Figure 1 (Sec. 3.2): run boundaries
// are flagged, a max-scan gives every byte the start of its run, a prefix sum
// of per-byte output counts gives output positions, and bytes are scattered.
// Inside a run, byte t (0-based) sits at u = t mod 255 of a piece of at most
// 255 bytes; it writes its own byte when u < 4, the byte at u = 3 also owns
// the slot of the piece's count byte, and the last byte of a piece writes the
// count u - 3 into that slot.  So every byte's output count depends only on
// u, never on the run's length, and long runs stay load-balanced.
//
// Tiles of RLE_TILE bytes never cross a block.  Pass A reduces each tile to
// (last run start, bytes before the first run start, output count of the
// bytes after it, CRC share); pass B scans tiles per block; pass C emits.
#include "common.hpp"
#include "internal.hpp"

namespace bzg {

constexpr int RITEMS = RLE_TILE / NT;  // 16 bytes per thread
// Most RLE1 output bytes of one tile: every byte emits at most 2 (the 4th
// of a piece: itself and the count slot).
constexpr uint32_t RLE_OUT_MAX = 2 * RLE_TILE;

struct RleTile {
  uint32_t last_bnd;  // last run start in the tile, +1 (0 = none)
  uint32_t lead;      // bytes before the tile's first run start
  uint32_t inner;     // output bytes of the bytes from the first run start on
  uint32_t crc;       // CRC share of the tile from a zero register (at the tile end)
};

__device__ __forceinline__ uint32_t rle_emit_count(uint32_t t) {
  uint32_t u = t % 255u;
  return u < 3 ? 1u : (u == 3 ? 2u : 0u);
}
// output bytes of the first x bytes of a run
__device__ __forceinline__ uint32_t rle_prefix(uint32_t x) {
  uint32_t r = x % 255u;
  return 5u * (x / 255u) + (r <= 3 ? r : 5u);
}

struct TileGeom {
  uint32_t b;       // block
  uint64_t base;    // block start in the input
  uint32_t n;       // block length
  uint32_t lo, hi;  // tile range inside the block
};

__device__ __forceinline__ TileGeom tile_geom(uint32_t t, const uint32_t* tile_blk, const uint32_t* blk_tile0,
                                              const uint64_t* blk_off) {
  TileGeom g;
  g.b = tile_blk[t];
  g.base = blk_off[g.b];
  g.n = (uint32_t)(blk_off[g.b + 1] - g.base);
  g.lo = (t - blk_tile0[g.b]) * RLE_TILE;
  g.hi = min(g.lo + RLE_TILE, g.n);
  return g;
}

// Loads this thread's RITEMS (16) bytes, as dwords, and the byte before them.
__device__ __forceinline__ void load_run(const uint8_t* s, const TileGeom& g, uint32_t p0, uint8_t* v,
                                         int& cnt, uint32_t& prev) {
  static_assert(RITEMS == 16, "one 16-byte span per thread");
  cnt = 0;
  prev = 0x100u;  // never equal to a byte
  if (p0 < g.hi) cnt = (int)min((uint32_t)RITEMS, g.hi - p0);
  if (p0 > 0 && p0 < g.hi) prev = s[g.base + p0 - 1];
  uint32_t w[4] = {0, 0, 0, 0};
  if (cnt) load16(s + g.base + p0, (uint32_t)cnt, w);
#pragma unroll
  for (int i = 0; i < RITEMS; i++) v[i] = i < cnt ? (uint8_t)(w[i >> 2] >> (8 * (i & 3))) : 0;
}

// 1 + the position of the last run start among this thread's bytes (0 when
// none starts here).  Loops run the full RITEMS with a mask so that v[] is
// indexed by constants and stays in registers.
__device__ __forceinline__ uint32_t last_run_start(const uint8_t* v, int cnt, uint32_t p0, uint32_t prev) {
  uint32_t lastb = 0, pv = prev;
#pragma unroll
  for (int i = 0; i < RITEMS; i++) {
    const bool st = (i < cnt) & ((p0 + i == 0) | (v[i] != pv));
    lastb = st ? p0 + i + 1 : lastb;
    pv = v[i];
  }
  return lastb;
}

// One tile of pass A: run starts, output counts and CRC share of tile t.
__device__ void rle1_tile(const uint8_t* __restrict__ s, uint32_t t, const uint32_t* tile_blk,
                          const uint32_t* blk_tile0, const uint64_t* blk_off, const uint32_t* crc_pow,
                          RleTile* tiles, uint32_t* sh, uint32_t* sx, uint32_t (*tab)[256]) {
  TileGeom g = tile_geom(t, tile_blk, blk_tile0, blk_off);
  const uint32_t p0 = g.lo + threadIdx.x * RITEMS;
  uint8_t v[RITEMS];
  int cnt;
  uint32_t prev;
  load_run(s, g, p0, v, cnt, prev);
  // CRC of this thread's bytes from a zero register, shifted to the tile end
  // (by a per-thread constant in full tiles)
  uint32_t reg = 0;
  if (cnt == RITEMS) {  // four bytes a step: 4 dependent lookups instead of 16
#pragma unroll
    for (int j = 0; j < RITEMS / 4; j++) {
      reg ^= ((uint32_t)v[4 * j] << 24) | ((uint32_t)v[4 * j + 1] << 16) | ((uint32_t)v[4 * j + 2] << 8) | v[4 * j + 3];
      reg = tab[3][reg >> 24] ^ tab[2][(reg >> 16) & 255u] ^ tab[1][(reg >> 8) & 255u] ^ tab[0][reg & 255u];
    }
  } else {
#pragma unroll
    for (int i = 0; i < RITEMS; i++)
      if (i < cnt) reg = (reg << 8) ^ tab[0][(reg >> 24) ^ v[i]];
  }
  uint32_t share = 0;
  if (cnt) {
    const uint32_t after = g.hi - (p0 + cnt);
    const uint32_t sft = (g.hi - g.lo == RLE_TILE) ? crc_pow[64 + threadIdx.x] : gf2_xpow8(after, crc_pow);
    share = gf2_mulmod(reg, sft);
  }
  // run starts
  uint32_t pv = prev;
  const uint32_t lastb = last_run_start(v, cnt, p0, prev);
  uint32_t incl = block_incl_max<uint32_t, NT>(lastb, sh, 0u);
  sx[threadIdx.x] = incl;
  __syncthreads();
  const uint32_t carry = threadIdx.x ? sx[threadIdx.x - 1] : 0u;
  const uint32_t tile_last = sx[NT - 1];
  // bytes before the tile's first run start; the others' output counts, all
  // 1 unless some byte is the 4th or later of its run
  uint32_t lead = 0, inner = 0, rs = carry, tmax = 0;
#pragma unroll
  for (int i = 0; i < RITEMS; i++) {
    const uint32_t p = p0 + i;
    const bool ok = i < cnt;
    rs = ok & ((p == 0) | (v[i] != pv)) ? p + 1 : rs;
    pv = v[i];
    lead += (ok & (rs == 0)) ? 1u : 0u;
    tmax = (ok & (rs != 0)) ? max(tmax, p - (rs - 1)) : tmax;
  }
  if (tmax < 3) {
    inner = (uint32_t)cnt - lead;
  } else {
    rs = carry;
    pv = prev;
#pragma unroll
    for (int i = 0; i < RITEMS; i++) {
      const uint32_t p = p0 + i;
      const bool ok = i < cnt;
      rs = ok & ((p == 0) | (v[i] != pv)) ? p + 1 : rs;
      pv = v[i];
      inner += (ok & (rs != 0)) ? rle_emit_count(p - (rs - 1)) : 0u;
    }
  }
  lead = block_sum<uint32_t, NT>(lead, sh);
  inner = block_sum<uint32_t, NT>(inner, sh);
  share = wave_xor(share);
  uint32_t w = threadIdx.x / BZG_WAVE;
  if (lane() == 0) sx[w] = share;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t c = 0;
    for (int i = 0; i < NT / BZG_WAVE; i++) c ^= sx[i];
    RleTile r;
    r.last_bnd = tile_last;
    r.lead = lead;
    r.inner = inner;
    r.crc = c;
    tiles[t] = r;
  }
}

// Pass A.  Persistent workgroups over the tiles (count *ntiles).
__global__ __launch_bounds__(NT) void k_rle1_tiles(const uint8_t* __restrict__ s, const uint32_t* __restrict__ ntiles,
                                                   const uint32_t* tile_blk, const uint32_t* blk_tile0,
                                                   const uint64_t* blk_off, const uint32_t* __restrict__ crc_tab,
                                                   const uint32_t* crc_pow, RleTile* tiles) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sx[NT];
  __shared__ uint32_t tab[4][256];  // slicing-by-4 tables (k + 1 byte steps)
#pragma unroll
  for (int k = 0; k < 4; k++) tab[k][threadIdx.x] = crc_tab[k * 256 + threadIdx.x];
  __syncthreads();
  for (TileLoop it = tile_loop(*ntiles); it.t < it.end; it.t += it.step) {
    rle1_tile(s, it.t, tile_blk, blk_tile0, blk_off, crc_pow, tiles, sh, sx, tab);
    __syncthreads();
  }
}

// One workgroup per block: scan its tiles.  Writes each tile's carried run
// start (+1, tile_rs) and output offset, the block's RLE1 length and CRC.
// The tile records are left as pass A wrote them.
__global__ __launch_bounds__(NT) void k_rle1_blocks(const uint32_t* blk_tile0, const uint64_t* blk_off,
                                                    const uint32_t* crc_pow, const RleTile* tiles,
                                                    uint32_t* tile_rs, uint32_t* tile_out, uint32_t* rle_n,
                                                    uint32_t* crc_out) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sx[NT];
  // the powers x^(8 * 2^j) in LDS: the shifts below take one per set bit of
  // a byte count, each read right before its use
  __shared__ uint32_t spw[64];
  if (threadIdx.x < 64) spw[threadIdx.x] = crc_pow[threadIdx.x];
  __syncthreads();
  const uint32_t b = blockIdx.x;
  const uint32_t t0 = blk_tile0[b], t1 = blk_tile0[b + 1];
  const uint32_t n = (uint32_t)(blk_off[b + 1] - blk_off[b]);
  uint32_t carry_rs = 0, carry_out = 0, x = 0;
  for (uint32_t c = t0; c < t1; c += NT) {
    uint32_t t = c + threadIdx.x;
    RleTile r = {0, 0, 0, 0};
    if (t < t1) r = tiles[t];
    uint32_t incl = block_incl_max<uint32_t, NT>(r.last_bnd, sh, 0u);
    sx[threadIdx.x] = incl;
    __syncthreads();
    uint32_t rs = threadIdx.x ? sx[threadIdx.x - 1] : 0u;
    rs = rs > carry_rs ? rs : carry_rs;
    uint32_t lo = (t - t0) * RLE_TILE;
    uint32_t e = 0;
    if (t < t1) {
      e = r.inner;
      if (r.lead) {  // the tile opens inside a run that started at rs-1
        uint32_t off = lo - (rs - 1);
        e += rle_prefix(off + r.lead) - rle_prefix(off);
      }
    }
    uint32_t tot;
    uint32_t ex = block_excl_sum<uint32_t, NT>(e, sh, &tot);
    if (t < t1) {
      tile_out[t] = carry_out + ex;
      tile_rs[t] = rs;  // run start carried into the tile (+1)
    }
    if (t < t1) x ^= gf2_mulmod(r.crc, gf2_xpow8((uint64_t)(n - min(lo + RLE_TILE, n)), spw));
    carry_out += tot;
    carry_rs = sx[NT - 1] > carry_rs ? sx[NT - 1] : carry_rs;
    __syncthreads();
  }
  uint32_t xa = wave_xor(x);
  if (lane() == 0) sx[threadIdx.x / BZG_WAVE] = xa;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t c = 0;
    for (int i = 0; i < NT / BZG_WAVE; i++) c ^= sx[i];
    uint32_t init = gf2_mulmod(0xFFFFFFFFu, gf2_xpow8((uint64_t)n, spw));
    crc_out[b] = ~(init ^ c);
    rle_n[b] = carry_out;
  }
}

// Walks one window [g.lo, g.hi) of a block with the carried run start
// `carry` (+1): computes each byte's output position.  MODE 0 writes the RLE1
// output at out + obase + tile_off.  MODE 1 measures: *res gets the window
// position after the last byte whose output ends at or before `limit`
// (counting from tile_off), the window's output total and its last run
// start (+1, 0 = none; the carry does not count).
struct WalkRes {
  uint32_t fit, tot, lastb;
};

template <int MODE>
__device__ void rle1_walk(const uint8_t* s, const TileGeom& g, uint32_t carry, uint32_t tile_off,
                          uint8_t* out, uint64_t obase, uint32_t limit, uint32_t* sh, uint32_t* sx,
                          WalkRes* res) {
  const uint32_t p0 = g.lo + threadIdx.x * RITEMS;
  // the byte after this thread's (read with the others; clamped when absent)
  const uint32_t pe = p0 + min((uint32_t)RITEMS, g.hi > p0 ? g.hi - p0 : 0u);
  const bool has_next = pe > p0 && pe < g.n;
  const uint8_t next = s[g.base + (has_next ? pe : 0u)];
  uint8_t v[RITEMS];
  int cnt;
  uint32_t prev;
  load_run(s, g, p0, v, cnt, prev);
  uint32_t pv = prev, e = 0;
  const uint32_t lastb = last_run_start(v, cnt, p0, prev);
  uint32_t incl = block_incl_max<uint32_t, NT>(lastb, sh, 0u);
  sx[threadIdx.x] = incl;
  __syncthreads();
  const uint32_t win_last = sx[NT - 1];
  uint32_t rs = threadIdx.x ? sx[threadIdx.x - 1] : 0u;
  rs = rs > carry ? rs : carry;
  uint32_t rs0 = rs;
  // Run offsets of this thread's bytes.  When none reaches 3 (no byte is the
  // 4th or later of a run: the common case outside long runs) every byte
  // emits itself and nothing else, and the per-byte piece logic is skipped.
  uint32_t tmax = 0;
#pragma unroll
  for (int i = 0; i < RITEMS; i++) {
    const uint32_t p = p0 + i;
    const bool ok = i < cnt;
    rs = ok & ((p == 0) | (v[i] != pv)) ? p + 1 : rs;
    pv = v[i];
    tmax = ok ? max(tmax, p - (rs - 1)) : tmax;
  }
  const bool plain = tmax < 3;
  if (plain) {
    e = (uint32_t)cnt;
  } else {
    rs = rs0;
    pv = prev;
#pragma unroll
    for (int i = 0; i < RITEMS; i++) {
      const uint32_t p = p0 + i;
      const bool ok = i < cnt;
      rs = ok & ((p == 0) | (v[i] != pv)) ? p + 1 : rs;
      pv = v[i];
      e += ok ? rle_emit_count(p - (rs - 1)) : 0u;
    }
  }
  uint32_t tot;
  // MODE 0 stages the tile's output in LDS (at the global dword alignment)
  // and writes it out coalesced.  A piece's count byte sits right after its
  // 4th byte; when the piece runs on into the next tile, that slot is this
  // tile's last output byte and the next tile writes it to global directly.
  __shared__ uint8_t sout[RLE_OUT_MAX + 4];
  __shared__ uint32_t s_skip;
  const uint64_t gbase = obase + tile_off;
  const uint32_t al = (uint32_t)(gbase & 3u);
  if (MODE == 0 && threadIdx.x == 0) s_skip = 0;
  uint32_t o = block_excl_sum<uint32_t, NT>(e, sh, &tot);  // local output position
  rs = rs0;
  pv = prev;
  uint32_t below = 0;
  if (plain) {
    if (MODE == 0) {
#pragma unroll
      for (int i = 0; i < RITEMS; i++)
        if (i < cnt) sout[al + o + i] = v[i];
    } else {
#pragma unroll
      for (int i = 0; i < RITEMS; i++) below += ((i < cnt) & (tile_off + o + i + 1 <= limit)) ? 1u : 0u;
    }
  } else {
#pragma unroll
    for (int i = 0; i < RITEMS; i++) {
      const uint32_t p = p0 + i;
      const bool ok = i < cnt;
      rs = ok & ((p == 0) | (v[i] != pv)) ? p + 1 : rs;
      pv = v[i];
      const uint32_t tt = p - (rs - 1);
      const uint32_t u = tt % 255u;
      const uint32_t ec = ok ? rle_emit_count(tt) : 0u;
      if (!ok) {
      } else if (MODE == 0) {
        if (u <= 3) sout[al + o] = v[i];
        // the byte after this one: the next of this thread's, else `next`
        const bool differs = (i + 1 < cnt) ? v[i + 1 < RITEMS ? i + 1 : i] != v[i] : (!has_next || next != v[i]);
        const bool last_of_piece = (u == 254) || differs;
        if (last_of_piece && u >= 3) {
          if (u == 3) sout[al + o + 1] = 0;
          else if (o > 0) sout[al + o - 1] = (uint8_t)(u - 3);
          else out[gbase - 1] = (uint8_t)(u - 3);  // slot in the previous tile's output
        }
        if (p + 1 == g.hi && u >= 3 && !last_of_piece) s_skip = 1;
      } else {
        if (tile_off + o + ec <= limit) below++;
      }
      o += ec;
    }
  }
  if (MODE == 0) {
    __syncthreads();
    const uint32_t len = tot - s_skip;
    const uint32_t nd = (al + len + 3) / 4;
    uint32_t* gw = (uint32_t*)(out + (gbase - al));
    const uint32_t* lw = (const uint32_t*)sout;
    for (uint32_t j = threadIdx.x; j < nd; j += NT) {
      if (4 * j >= al && 4 * j + 4 <= al + len) {
        gw[j] = lw[j];
      } else {
        for (uint32_t q = max(4 * j, al); q < min(4 * j + 4, al + len); q++) out[gbase - al + q] = sout[q];
      }
    }
  }
  if (MODE == 1) {
    below = block_sum<uint32_t, NT>(below, sh);
    if (threadIdx.x == 0) {
      res->fit = g.lo + below;
      res->tot = tot;
      res->lastb = win_last;
    }
    __syncthreads();
  }
}

// Pass C.  Persistent workgroups over the tiles: every tile writes its RLE1
// output at its block's offset roff[b] plus the tile's output offset.
__global__ __launch_bounds__(NT) void k_rle1_emit(const uint8_t* __restrict__ s, const uint32_t* __restrict__ ntiles,
                                                  const uint32_t* tile_blk, const uint32_t* blk_tile0,
                                                  const uint64_t* blk_off, const uint32_t* tile_rs,
                                                  const uint32_t* tile_out, const uint32_t* roff,
                                                  uint8_t* __restrict__ out) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sx[NT];
  for (TileLoop it = tile_loop(*ntiles); it.t < it.end; it.t += it.step) {
    const uint32_t t = it.t;
    TileGeom g = tile_geom(t, tile_blk, blk_tile0, blk_off);
    rle1_walk<0>(s, g, tile_rs[t], tile_out[t], out, roff[g.b], 0, sh, sx, nullptr);
    __syncthreads();
  }
}

// Most input bytes whose fresh RLE1 output (a run starting at the first of
// them) fits in L bytes: 255 per 5 output bytes, then up to 3 literal bytes.
__device__ __forceinline__ uint32_t run_fit(uint32_t L) { return 255u * (L / 5u) + min(L % 5u, 3u); }

// Block cutting.  One workgroup per input block k: the block's pieces are
// the longest prefixes whose own RLE1 output fits in L bytes, one after
// another (RLE1 restarts at every piece, so a run that crosses a cut starts
// afresh).  Piece j of block k goes to slot slot_base[k] + j
// (slot_in[slot] = its first input byte, relative); slots the block does not
// need get empty ranges at the block end.  Inputs are the block's whole-
// stream tile records (pass A and B over the input blocks that may need
// cutting; a block with one slot has no tiles, RLE1 length 0, and keeps its
// whole range): tile_out[t] is
// the output position P of the tile's first byte and P is what the block's
// RLE1 stream has written before a byte.
//
// A piece starting at s0 follows the whole stream once its first run ends
// (after that, RLE1 output only depends on the bytes): with M a position
// past that run, the piece's output up to e >= M is F(M) + P(e) - P(M), so
// the cut is where the whole stream passes L - F(M) + P(M).  The first window
// (up to the next tile boundary) is walked afresh; a run that outlasts it is
// measured from the tile records (tiles with no run start lie inside it).
__global__ __launch_bounds__(NT) void k_rle1_split(const uint8_t* __restrict__ s, const uint64_t* __restrict__ in_off,
                                                   uint32_t n_in, const uint32_t* __restrict__ in_tile0,
                                                   const RleTile* __restrict__ tiles,
                                                   const uint32_t* __restrict__ tile_rs,
                                                   const uint32_t* __restrict__ tile_out,
                                                   const uint32_t* __restrict__ rle_n,
                                                   const uint32_t* __restrict__ slot_base, uint32_t nslot, uint32_t L,
                                                   uint64_t* __restrict__ slot_in, uint32_t* __restrict__ err) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sx[NT];
  __shared__ WalkRes wr;
  __shared__ uint32_t s_t2;
  const uint32_t k = blockIdx.x;
  const uint64_t base = in_off[k];
  const uint32_t n = (uint32_t)(in_off[k + 1] - base);
  const uint32_t sb = slot_base[k], np = slot_base[k + 1] - sb;
  const uint32_t t0 = in_tile0[k], t1 = in_tile0[k + 1];
  if (k + 1 == n_in && threadIdx.x == 0) slot_in[nslot] = in_off[n_in];
  if (np == 0) return;  // an empty block has no slot
  TileGeom g;
  g.b = k;
  g.base = base;
  g.n = n;
  uint32_t j = 0, s0 = 0;
  const uint32_t total = rle_n[k];
  for (;;) {
    if (threadIdx.x == 0) slot_in[sb + j] = base + s0;
    j++;
    if (s0 == 0 && total <= L) break;  // the whole block fits
    // the cut of the piece starting at s0 (e == n: the rest fits)
    uint32_t e;
    const uint32_t t = t0 + s0 / RLE_TILE;
    const uint32_t W = min((s0 / RLE_TILE + 1) * RLE_TILE, n);
    g.lo = s0;
    g.hi = W;
    rle1_walk<1>(s, g, s0 + 1, 0, nullptr, 0, L, sh, sx, &wr);
    const WalkRes a = wr;
    if (a.fit < W) {
      e = a.fit;
    } else if (W == n) {
      e = n;
    } else {
      uint32_t F, P, tM;
      bool done = false;
      e = n;
      if (a.lastb > s0 + 1) {  // the first run ends inside the window
        F = a.tot;
        P = tile_out[t + 1];
        tM = t + 1;
      } else {  // it runs on: find the next tile with a run start
        if (threadIdx.x == 0) s_t2 = t1;
        __syncthreads();
        for (uint32_t c = t + 1; c < t1; c += NT) {
          const uint32_t q = c + threadIdx.x;
          const bool hit = q < t1 && tiles[min(q, t1 - 1)].last_bnd != 0;
          const uint64_t m = __ballot(hit);
          if (m && lane() == 0) atomicMin(&s_t2, c + (threadIdx.x & ~63u) + (uint32_t)(__ffsll((long long)m) - 1));
          __syncthreads();
          const bool found = s_t2 < t1;
          __syncthreads();  // every thread has read s_t2 before any writes it again
          if (found) break;
        }
        const uint32_t t2 = s_t2;
        const uint32_t r1 = t2 < t1 ? (t2 - t0) * RLE_TILE + tiles[t2].lead : n;
        F = rle_prefix(r1 - s0);
        if (F > L) {
          e = s0 + run_fit(L);
          done = true;
        } else if (r1 == n) {
          e = n;
          done = true;
        } else {
          const uint32_t lo2 = (t2 - t0) * RLE_TILE, off = lo2 - (tile_rs[t2] - 1);
          P = tile_out[t2] + rle_prefix(off + tiles[t2].lead) - rle_prefix(off);
          tM = t2;
        }
      }
      if (!done) {
        const uint32_t T = L - F + P;  // whole-stream positions up to T fit
        if (total <= T) {
          e = n;
        } else {
          uint32_t lo = tM, hi = t1 - 1;  // first tile whose end passes T
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            const uint32_t end = mid + 1 < t1 ? tile_out[mid + 1] : total;
            if (end > T) hi = mid; else lo = mid + 1;
          }
          g.lo = (lo - t0) * RLE_TILE;
          g.hi = min(g.lo + RLE_TILE, n);
          rle1_walk<1>(s, g, tile_rs[lo], tile_out[lo], nullptr, 0, T, sh, sx, &wr);
          e = wr.fit;
        }
      }
    }
    if (e >= n) break;
    if (e <= s0 || j >= np) {  // no progress or more pieces than slots: cannot happen
      if (threadIdx.x == 0) atomicOr(err, ERR_BOUND);
      break;
    }
    s0 = e;
  }
  for (uint32_t q = j + threadIdx.x; q < np; q += NT) slot_in[sb + q] = base + n;
}

hipError_t rle1_tiles(const uint8_t* s, uint32_t grid, const uint32_t* ntiles, const uint32_t* tile_blk,
                      const uint32_t* blk_tile0, const uint64_t* blk_off, const uint32_t* crc_tab,
                      const uint32_t* crc_pow, void* tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_rle1_tiles, dim3(grid), dim3(NT), 0, st, s, ntiles, tile_blk, blk_tile0, blk_off, crc_tab,
                     crc_pow, (RleTile*)tiles);
  return hipGetLastError();
}

hipError_t rle1_blocks(uint32_t nb, const uint32_t* blk_tile0, const uint64_t* blk_off, const uint32_t* crc_pow,
                       const void* tiles, uint32_t* tile_rs, uint32_t* tile_out, uint32_t* rle_n, uint32_t* crc,
                       hipStream_t st) {
  if (nb) hipLaunchKernelGGL(k_rle1_blocks, dim3(nb), dim3(NT), 0, st, blk_tile0, blk_off, crc_pow,
                             (const RleTile*)tiles, tile_rs, tile_out, rle_n, crc);
  return hipGetLastError();
}

hipError_t rle1_emit(const uint8_t* s, uint32_t grid, const uint32_t* ntiles, const uint32_t* tile_blk,
                     const uint32_t* blk_tile0, const uint64_t* blk_off, const uint32_t* tile_rs,
                     const uint32_t* tile_out, const uint32_t* roff, uint8_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rle1_emit, dim3(grid), dim3(NT), 0, st, s, ntiles, tile_blk, blk_tile0, blk_off, tile_rs,
                     tile_out, roff, out);
  return hipGetLastError();
}

hipError_t rle1_split(const uint8_t* s, const uint64_t* in_off, uint32_t n_in, const uint32_t* in_tile0,
                      const void* tiles, const uint32_t* tile_rs, const uint32_t* tile_out, const uint32_t* rle_n,
                      const uint32_t* slot_base, uint32_t nslot, uint32_t L, uint64_t* slot_in, uint32_t* err,
                      hipStream_t st) {
  if (n_in) hipLaunchKernelGGL(k_rle1_split, dim3(n_in), dim3(NT), 0, st, s, in_off, n_in, in_tile0,
                               (const RleTile*)tiles, tile_rs, tile_out, rle_n, slot_base, nslot, L, slot_in, err);
  return hipGetLastError();
}

size_t rle_tile_bytes() { return sizeof(RleTile); }

}  // namespace bzg
