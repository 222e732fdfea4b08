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

// Pass A.  One workgroup per tile: tile ids[blockIdx.x], or every tile when
// ids is null.
__global__ __launch_bounds__(NT) void k_rle1_tiles(const uint8_t* __restrict__ s, const uint32_t* __restrict__ ids,
                                                   const uint32_t* tile_blk, const uint32_t* blk_tile0,
                                                   const uint64_t* blk_off, const uint32_t* __restrict__ crc_tab,
                                                   const uint32_t* crc_pow, RleTile* tiles) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sx[NT];
  __shared__ uint32_t tab[4][256];  // slicing-by-4 tables (k + 1 byte steps)
#pragma unroll
  for (int k = 0; k < 4; k++) tab[k][threadIdx.x] = crc_tab[k * 256 + threadIdx.x];
  const uint32_t t = ids ? ids[blockIdx.x] : blockIdx.x;
  TileGeom g = tile_geom(t, tile_blk, blk_tile0, blk_off);
  const uint32_t p0 = g.lo + threadIdx.x * RITEMS;
  uint8_t v[RITEMS];
  int cnt;
  uint32_t prev;
  load_run(s, g, p0, v, cnt, prev);
  __syncthreads();
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

// Walks one tile with the carried run start: computes each byte's output
// position.  mode 0 writes RLE1 output at out + out_base[b]; mode 1 counts the
// bytes whose output ends at or before `limit` (the block is cut there).
template <int MODE>
__device__ void rle1_walk(const uint8_t* s, const TileGeom& g, uint32_t carry, uint32_t tile_off,
                          uint8_t* out, uint64_t obase, uint32_t limit, uint32_t* sh, uint32_t* sx,
                          uint32_t* count_out) {
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
    if (threadIdx.x == 0) *count_out = g.lo + below;
  }
}

__global__ __launch_bounds__(NT) void k_rle1_emit(const uint8_t* __restrict__ s, const uint32_t* tile_blk,
                                                  const uint32_t* blk_tile0, const uint64_t* blk_off,
                                                  const uint32_t* tile_rs, const uint32_t* tile_out,
                                                  const uint64_t* out_base, uint8_t* __restrict__ out) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sx[NT];
  const uint32_t t = blockIdx.x;
  TileGeom g = tile_geom(t, tile_blk, blk_tile0, blk_off);
  rle1_walk<0>(s, g, tile_rs[t], tile_out[t], out, out_base[g.b], 0, sh, sx, nullptr);
}

// Tile records carried over from the previous plan: dst[t] = src[from[t]]
// where from[t] is not ~0.
__global__ __launch_bounds__(NT) void k_tile_copy(uint32_t n, const uint32_t* __restrict__ from,
                                                  const RleTile* __restrict__ src, RleTile* __restrict__ dst) {
  const uint32_t t = blockIdx.x * NT + threadIdx.x;
  if (t < n && from[t] != ~0u) dst[t] = src[from[t]];
}

// One workgroup per oversized block: the length of the longest input prefix
// whose RLE1 output fits in `limit` bytes.
__global__ __launch_bounds__(NT) void k_rle1_cut(const uint8_t* __restrict__ s, const uint32_t* blk_ids,
                                                 const uint32_t* blk_tile0, const uint64_t* blk_off,
                                                 const uint32_t* tile_rs, const uint32_t* tile_out,
                                                 uint32_t limit, uint32_t* cut) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sx[NT];
  __shared__ uint32_t tsel;
  const uint32_t b = blk_ids[blockIdx.x];
  const uint32_t t0 = blk_tile0[b], t1 = blk_tile0[b + 1];
  if (threadIdx.x == 0) {  // last tile whose output starts at or below the limit
    uint32_t lo = t0, hi = t1 - 1;
    while (lo < hi) {
      uint32_t mid = (lo + hi + 1) / 2;
      if (tile_out[mid] <= limit) lo = mid; else hi = mid - 1;
    }
    tsel = lo;
  }
  __syncthreads();
  const uint32_t t = tsel;
  TileGeom g;
  g.b = b;
  g.base = blk_off[b];
  g.n = (uint32_t)(blk_off[b + 1] - g.base);
  g.lo = (t - t0) * RLE_TILE;
  g.hi = min(g.lo + RLE_TILE, g.n);
  rle1_walk<1>(s, g, tile_rs[t], tile_out[t], nullptr, 0, limit, sh, sx, &cut[blockIdx.x]);
}

hipError_t rle1_tiles(const uint8_t* s, uint32_t nlaunch, const uint32_t* ids, const uint32_t* tile_blk,
                      const uint32_t* blk_tile0, const uint64_t* blk_off, const uint32_t* crc_tab,
                      const uint32_t* crc_pow, void* tiles, hipStream_t st) {
  if (nlaunch) hipLaunchKernelGGL(k_rle1_tiles, dim3(nlaunch), dim3(NT), 0, st, s, ids, tile_blk, blk_tile0, blk_off,
                                  crc_tab, crc_pow, (RleTile*)tiles);
  return hipGetLastError();
}

hipError_t rle1_tile_copy(uint32_t n, const uint32_t* from, const void* src, void* dst, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_tile_copy, dim3((n + NT - 1) / NT), dim3(NT), 0, st, n, from, (const RleTile*)src,
                            (RleTile*)dst);
  return hipGetLastError();
}

hipError_t rle1_blocks(uint32_t nb, const uint32_t* blk_tile0, const uint64_t* blk_off, const uint32_t* crc_pow,
                       const void* tiles, uint32_t* tile_rs, uint32_t* tile_out, uint32_t* rle_n, uint32_t* crc,
                       hipStream_t st) {
  if (nb) hipLaunchKernelGGL(k_rle1_blocks, dim3(nb), dim3(NT), 0, st, blk_tile0, blk_off, crc_pow,
                             (const RleTile*)tiles, tile_rs, tile_out, rle_n, crc);
  return hipGetLastError();
}

hipError_t rle1_emit(const uint8_t* s, uint32_t ntiles, const uint32_t* tile_blk, const uint32_t* blk_tile0,
                     const uint64_t* blk_off, const uint32_t* tile_rs, const uint32_t* tile_out,
                     const uint64_t* out_base, uint8_t* out, hipStream_t st) {
  if (ntiles) hipLaunchKernelGGL(k_rle1_emit, dim3(ntiles), dim3(NT), 0, st, s, tile_blk, blk_tile0, blk_off, tile_rs,
                                 tile_out, out_base, out);
  return hipGetLastError();
}

hipError_t rle1_cut(const uint8_t* s, uint32_t ncut, const uint32_t* blk_ids, const uint32_t* blk_tile0,
                    const uint64_t* blk_off, const uint32_t* tile_rs, const uint32_t* tile_out, uint32_t limit,
                    uint32_t* cut, hipStream_t st) {
  if (ncut) hipLaunchKernelGGL(k_rle1_cut, dim3(ncut), dim3(NT), 0, st, s, blk_ids, blk_tile0, blk_off, tile_rs,
                               tile_out, limit, cut);
  return hipGetLastError();
}

size_t rle_tile_bytes() { return sizeof(RleTile); }

}  // namespace bzg
