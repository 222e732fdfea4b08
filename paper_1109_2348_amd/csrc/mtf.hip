// Move-to-front (Sec. 3.3) with RUNA/RUNB zero-run coding, chunked.
//
// The paper parallelises one MTF step over the recency stack: every
// processor checks one stack slot and the match is unique.  Here a wave64
// holds the 256-slot stack, four slots per lane, and one ballot per slot
// column finds the symbol.  That alone is serial over the block, so blocks
// are cut into chunks and the stack is carried between them: after a chunk X
// the stack is D_X followed by the incoming stack with D_X removed, where D_X
// lists X's distinct symbols by last occurrence, latest first.  That map
// composes associatively, so chunk summaries are computed in parallel, a
// per-block scan yields each chunk's incoming stack, and all chunks re-run
// MTF in parallel.
//
// MTF index 0 at row j means L[j] == L[j-1] (at the block's first row: L[0]
// is the smallest in-use byte), so zero runs -- and the RUNA/RUNB symbol
// counts -- are known from L alone.  A chunk's zero-run summary
// (leading zeros, trailing zeros, all-zero flag, digits of runs closed
// inside, nonzero count) forms a monoid; the scan turns it into every
// chunk's output offset.  A run is coded where it ends.
#include "common.hpp"
#include "internal.hpp"

namespace bzg {

// Chunk length: MTF_CHUNK rows, or MTF_CHUNK_SMALL when a call holds so few
// chunks that the long per-chunk chains would leave the GPU idle.
constexpr uint32_t MTF_CHUNK_SMALL = 2048;
constexpr uint32_t MTF_FEW_CHUNKS = 64;

struct ZSum {
  uint32_t lz, tz, inner, nnz, len, all;
};

__device__ __forceinline__ uint32_t run_digits(uint32_t r) { return 31u - __clz(r + 1u); }

__device__ __forceinline__ ZSum zcombine(const ZSum& a, const ZSum& b) {
  ZSum r;
  r.len = a.len + b.len;
  if (a.all && b.all) {
    r = a;
    r.len = a.len + b.len;
    r.lz = r.tz = r.len;
    return r;
  }
  r.all = 0;
  if (a.all) {
    r.lz = a.len + b.lz;
    r.tz = b.tz;
    r.inner = b.inner;
    r.nnz = b.nnz;
  } else if (b.all) {
    r.lz = a.lz;
    r.tz = a.tz + b.len;
    r.inner = a.inner;
    r.nnz = a.nnz;
  } else {
    r.lz = a.lz;
    r.tz = b.tz;
    r.inner = a.inner + b.inner + run_digits(a.tz + b.lz);
    r.nnz = a.nnz + b.nnz;
  }
  return r;
}

// zcombine over the wave in lane order; lane 0 gets the result.
__device__ __forceinline__ ZSum zreduce_wave(ZSum v) {
  const uint32_t l = lane();
#pragma unroll
  for (int d = 1; d < BZG_WAVE; d <<= 1) {
    ZSum o;
    o.lz = __shfl_down(v.lz, d, BZG_WAVE);
    o.tz = __shfl_down(v.tz, d, BZG_WAVE);
    o.inner = __shfl_down(v.inner, d, BZG_WAVE);
    o.nnz = __shfl_down(v.nnz, d, BZG_WAVE);
    o.len = __shfl_down(v.len, d, BZG_WAVE);
    o.all = __shfl_down(v.all, d, BZG_WAVE);
    if ((l & (2 * d - 1)) == 0 && l + d < BZG_WAVE) v = zcombine(v, o);
  }
  return v;
}

struct ChunkGeom {
  uint32_t b, lo, hi, blo, bhi;  // block, chunk rows [lo,hi), block rows [blo,bhi)
  bool last;
};

__device__ __forceinline__ ChunkGeom chunk_geom(uint32_t c, const uint32_t* chunk_blk, const uint32_t* blk_chunk0,
                                                const uint32_t* off, uint32_t ch) {
  ChunkGeom g;
  g.b = chunk_blk[c];
  g.blo = off[g.b];
  g.bhi = off[g.b + 1];
  g.lo = g.blo + (c - blk_chunk0[g.b]) * ch;
  g.hi = min(g.lo + ch, g.bhi);
  g.last = (c + 1 == blk_chunk0[g.b + 1]);
  return g;
}

// This thread's MI consecutive rows from r0 (those below hi) as dwords;
// returns how many are valid.
template <int MI>
__device__ __forceinline__ uint32_t load_rows(const uint8_t* __restrict__ L, uint32_t r0, uint32_t hi,
                                              uint32_t w[MI / 4]) {
  static_assert(MI % 8 == 0, "whole 8-byte spans per thread");
  const uint32_t cnt = r0 < hi ? min((uint32_t)MI, hi - r0) : 0u;
#pragma unroll
  for (int j = 0; j < MI / 4; j++) w[j] = 0;
#pragma unroll
  for (uint32_t h = 0; h < (uint32_t)MI; h += 16) {
    if (cnt > h) {
      uint32_t t[4];
      load16(L + r0 + h, min(cnt - h, (uint32_t)min(MI - (int)h, 16)), t);
#pragma unroll
      for (int j = 0; j < 4; j++)
        if ((int)(h / 4) + j < MI / 4) w[h / 4 + j] = t[j];
    }
  }
  return cnt;
}

// Per chunk: D_X (distinct bytes by last occurrence, latest first), the
// zero-run summary of its rows -- without the block's first row, whose MTF
// index depends on the whole block's in-use set and is added by k_mtf_scan --
// and the chunk's in-use bitmap (8 words; k_mtf_scan ORs a block's chunks).
template <uint32_t CH>
__device__ void mtf_state_chunk(uint32_t c, const uint8_t* __restrict__ L, const uint32_t* chunk_blk,
                                const uint32_t* blk_chunk0, const uint32_t* off, uint32_t* __restrict__ chunk_inuse,
                                uint8_t* __restrict__ chunk_D, uint32_t* __restrict__ chunk_nD,
                                ZSum* __restrict__ chunk_sum) {
  constexpr int MITEMS = CH / NT;  // rows per thread
  constexpr uint32_t PW = CH / 32;  // words of the last-occurrence position bitmap
  __shared__ uint32_t last[256];
  __shared__ uint32_t pbits[PW], psuf[PW];
  __shared__ uint32_t ssh[NT / BZG_WAVE + 1];
  __shared__ ZSum wsum[NT / BZG_WAVE];
  __shared__ uint32_t s_nd;
  ChunkGeom g = chunk_geom(c, chunk_blk, blk_chunk0, off, CH);
  last[threadIdx.x] = 0;
  for (uint32_t i = threadIdx.x; i < PW; i += NT) pbits[i] = 0;
  if (threadIdx.x == 0) s_nd = 0;
  __syncthreads();
  // rows [lo + t*MITEMS, +MITEMS): last occurrences and the zero-run summary
  const uint32_t r0 = g.lo + threadIdx.x * MITEMS;
  uint8_t v[MITEMS];
  uint32_t prev = 0x100u;
  if (r0 < g.hi && r0 > g.blo) prev = L[r0 - 1];
  uint32_t w[MITEMS / 4];
  load_rows<MITEMS>(L, r0, g.hi, w);
  ZSum s = {0, 0, 0, 0, 0, 1};
#pragma unroll
  for (int i = 0; i < MITEMS; i++) {
    uint32_t k = r0 + i;
    if (k < g.hi) {
      v[i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
      if (k != g.blo) {
        ZSum e;
        if (v[i] == prev) e = {1, 1, 0, 0, 1, 1};
        else e = {0, 0, 0, 1, 1, 0};
        s = zcombine(s, e);
      }
      prev = v[i];
    }
  }
  // last occurrence: scan own rows backwards, report each byte once
  {
    uint32_t seen[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = MITEMS - 1; i >= 0; i--) {  // unrolled: v[] indexed by constants
      uint32_t k = r0 + i;
      if (k >= g.hi) continue;
      uint32_t x = v[i];
      uint32_t bit = 1u << (x & 31);
      uint32_t word = 0;
#pragma unroll
      for (int j = 0; j < 8; j++) word |= ((x >> 5) == (uint32_t)j) ? seen[j] : 0u;
      if (!(word & bit)) {
#pragma unroll
        for (int j = 0; j < 8; j++) seen[j] |= ((x >> 5) == (uint32_t)j) ? bit : 0u;
        atomicMax(&last[x], k - g.lo + 1);
      }
    }
  }
  __syncthreads();
  // D_X: present bytes by last occurrence, latest first
  {
    uint32_t x = threadIdx.x;
    uint32_t lx = last[x];
    const uint64_t present = __ballot(lx != 0);  // bytes 64w .. 64w+63
    static_assert(NT == 4 * BZG_WAVE, "four waves cover the 256 bytes");
    if (lane() == 0) {
      const uint32_t wv = threadIdx.x / BZG_WAVE;
      chunk_inuse[(size_t)c * 8 + 2 * wv] = (uint32_t)present;
      chunk_inuse[(size_t)c * 8 + 2 * wv + 1] = (uint32_t)(present >> 32);
    }
    // rank = present bytes whose last occurrence is later: the positions
    // (distinct, 1..CH) go into a bitmap, and a byte's rank is the number of
    // set bits above its own (suffix counts per word from one scan)
    if (lx) atomicOr(&pbits[(lx - 1u) >> 5], 1u << ((lx - 1u) & 31u));
    __syncthreads();
    static_assert(PW <= NT, "one bitmap word per thread");
    const uint32_t wc = threadIdx.x < PW ? (uint32_t)__popc(pbits[PW - 1u - threadIdx.x]) : 0u;
    uint32_t all;
    const uint32_t above = block_excl_sum<uint32_t, NT>(wc, ssh, &all);  // bits in words after it
    if (threadIdx.x < PW) psuf[PW - 1u - threadIdx.x] = above;
    __syncthreads();
    if (lx) {
      const uint32_t q = lx - 1u;
      const uint32_t r = psuf[q >> 5] + (uint32_t)__popc((pbits[q >> 5] >> (q & 31u)) >> 1);
      chunk_D[(size_t)c * 256 + r] = (uint8_t)x;
      atomicAdd(&s_nd, 1u);
    }
  }
  {
    const ZSum t = zreduce_wave(s);  // this wave's rows, in order
    if (lane() == 0) wsum[threadIdx.x / BZG_WAVE] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ZSum t = wsum[0];
    for (int i = 1; i < NT / BZG_WAVE; i++) t = zcombine(t, wsum[i]);
    chunk_sum[c] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) chunk_nD[c] = s_nd;
}

// Persistent workgroups over the *n_chunks chunks (at most cap).
template <uint32_t CH>
__global__ __launch_bounds__(NT) void k_mtf_state(const uint8_t* __restrict__ L, const uint32_t* chunk_blk,
                                                  const uint32_t* blk_chunk0, const uint32_t* off,
                                                  uint32_t* __restrict__ chunk_inuse, uint8_t* __restrict__ chunk_D,
                                                  uint32_t* __restrict__ chunk_nD, ZSum* __restrict__ chunk_sum,
                                                  const uint32_t* __restrict__ n_chunks, uint32_t cap) {
  for (TileLoop it = tile_loop(min(*n_chunks, cap)); it.t < it.end; it.t += it.step) {
    mtf_state_chunk<CH>(it.t, L, chunk_blk, blk_chunk0, off, chunk_inuse, chunk_D, chunk_nD, chunk_sum);
    __syncthreads();
  }
}

// Chunk summaries compose associatively: after chunk X the stack is D_X
// followed by the rest of the incoming stack in order, and after X then Y it
// is D_Y, then D_X minus D_Y, then the rest; zero-run summaries compose by
// zcombine.  So a block's chunks are scanned by SW waves in three steps:
// each wave composes the summaries of one contiguous range of chunks; one
// wave turns those into every range's incoming stack and prefix summary;
// each wave then walks its range from there.  The serial depth is about
// 2 * chunks / SW + SW steps instead of chunks: 16 waves when blocks hold
// many chunks, 8 otherwise.
constexpr int SCAN_WAVES = 8, SCAN_WAVES_LARGE = 16;
constexpr uint32_t SCAN_LARGE_CHUNKS = 64;  // average chunks per block from which 16 waves pay

// Between the steps of one wave's serial work in LDS (no workgroup barrier:
// the waves run independent loops).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The wave's stack e (slot j*64 + lane; 0x100 = empty) becomes D (nd bytes,
// dx) followed by the bytes of e not in D, in their order, then empty slots.
// e may be partial (a composed summary) and D may hold bytes e lacks.  mem
// (256, zero on entry and exit) and tmp (256) are this wave's LDS.
__device__ __forceinline__ void stack_front(uint32_t e[4], const uint32_t dx[4], uint32_t nd, uint8_t* mem,
                                            uint32_t* tmp) {
  const uint32_t l = lane();
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int j = 0; j < 4; j++)
    if ((uint32_t)(j * 64) + l < nd) mem[dx[j]] = 1;
  wave_sync();
  uint32_t mb[4];  // membership reads first, all together
#pragma unroll
  for (int j = 0; j < 4; j++) mb[j] = mem[e[j] & 255u];
  bool keep[4];
  uint64_t km[4];
#pragma unroll
  for (int j = 0; j < 4; j++) {
    keep[j] = (e[j] < 256u) & (mb[j] == 0u);
    km[j] = __ballot(keep[j]);
  }
#pragma unroll
  for (int j = 0; j < 4; j++) tmp[j * 64 + l] = (uint32_t)(j * 64) + l < nd ? dx[j] : 0x100u;
  wave_sync();
  uint32_t before = 0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    if (keep[j]) tmp[nd + before + (uint32_t)__popcll(km[j] & lt)] = e[j];
    before += (uint32_t)__popcll(km[j]);
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < 4; j++) e[j] = tmp[j * 64 + l];
#pragma unroll
  for (int j = 0; j < 4; j++)
    if ((uint32_t)(j * 64) + l < nd) mem[dx[j]] = 0;
  wave_sync();
}

__device__ __forceinline__ uint32_t zs_carry(const ZSum& p) { return p.all ? p.len : p.tz; }
__device__ __forceinline__ uint32_t zs_out(const ZSum& p) {
  return p.all ? 0u : p.nnz + p.inner + run_digits(p.lz);
}

// One workgroup of SW waves per block.  Writes every chunk's incoming
// stack, carried zero count and output offset, and the block's symbol count.
template <int SW>
__global__ __launch_bounds__(SW * BZG_WAVE) void k_mtf_scan(
    const uint32_t* blk_chunk0, const uint32_t* __restrict__ chunk_inuse, uint32_t* __restrict__ inuse,
    uint32_t* __restrict__ freq, uint32_t* __restrict__ err, const uint8_t* __restrict__ L,
    const uint32_t* __restrict__ off, const uint8_t* __restrict__ chunk_D, const uint32_t* __restrict__ chunk_nD,
    const ZSum* __restrict__ chunk_sum, uint8_t* __restrict__ chunk_list, uint32_t* __restrict__ chunk_carry,
    uint32_t* __restrict__ chunk_out, uint32_t* __restrict__ nsyms) {
  __shared__ uint32_t tmp[SW][256];
  __shared__ uint8_t mem[SW][256];
  __shared__ uint8_t gD[SW][256];  // each range's composed D (then incoming stack)
  __shared__ uint32_t gn[SW];
  __shared__ ZSum gz[SW];
  const uint32_t b = blockIdx.x;
  const uint32_t l = lane(), w = threadIdx.x / BZG_WAVE;
  __shared__ uint32_t sbm[8];
  const uint32_t c0 = blk_chunk0[b], c1 = blk_chunk0[b + 1], nc = c1 - c0;
  // the block's in-use bitmap: wave w ORs word w over the block's chunks
  // (and publishes it); the block's symbol counts start from zero
  static_assert(SW >= 8, "one wave per bitmap word");
  if (w < 8) {
    uint32_t x = 0;
#pragma unroll 4
    for (uint32_t c = c0 + l; c < c1; c += BZG_WAVE) x |= chunk_inuse[(size_t)c * 8 + w];
    x = wave_or(x);
    if (l == 0) {
      sbm[w] = x;
      inuse[b * 8 + w] = x;
    }
  }
  for (uint32_t i = threadIdx.x; i < (uint32_t)MAXA; i += SW * BZG_WAVE) freq[(size_t)b * MAXA + i] = 0;
  __syncthreads();
  uint32_t bm[8], nu = 0;
  for (int j = 0; j < 8; j++) {
    bm[j] = sbm[j];
    nu += __popc(bm[j]);
  }
#pragma unroll
  for (int j = 0; j < 4; j++) mem[w][j * 64 + l] = 0;
  // the block's first row: MTF index 0 exactly when it holds the smallest
  // in-use byte (the front of the initial stack)
  uint32_t minb = 0;
  for (int j = 7; j >= 0; j--)
    if (bm[j]) minb = j * 32 + (__ffs(bm[j]) - 1);
  const bool row0_zero = nc && L[off[b]] == minb;
  const ZSum e0 = row0_zero ? ZSum{1, 1, 0, 0, 1, 1} : ZSum{0, 0, 0, 1, 1, 0};
  const ZSum zid = {0, 0, 0, 0, 0, 1};
  // this wave's chunk range
  const uint32_t per = (nc + SW - 1) / SW;
  const uint32_t r0 = c0 + min(w * per, nc), r1 = c0 + min(w * per + per, nc);
  auto load_d = [&](uint32_t c, uint32_t dx[4], uint32_t& nd, ZSum& z) {
    nd = chunk_nD[c];
#pragma unroll
    for (int j = 0; j < 4; j++) dx[j] = (uint32_t)(j * 64) + l < nd ? chunk_D[(size_t)c * 256 + j * 64 + l] : 0u;
    z = chunk_sum[c];
    if (c == c0) z = zcombine(e0, z);
  };
  // step 1: compose the range's summaries (the next chunk's loaded ahead)
  {
    uint32_t e[4] = {0x100u, 0x100u, 0x100u, 0x100u};
    ZSum zg = zid;
    uint32_t dn[4] = {0, 0, 0, 0}, ndn = 0;
    ZSum zn = zid;
    if (r0 < r1) load_d(r0, dn, ndn, zn);
    for (uint32_t c = r0; c < r1; c++) {
      uint32_t dx[4] = {dn[0], dn[1], dn[2], dn[3]};
      const uint32_t nd = ndn;
      const ZSum z = zn;
      if (c + 1 < r1) load_d(c + 1, dn, ndn, zn);
      stack_front(e, dx, nd, mem[w], tmp[w]);
      zg = zcombine(zg, z);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) gD[w][j * 64 + l] = (uint8_t)(e[j] & 255u);
    uint32_t cnt = 0;  // the composed D's length: its non-empty slots
#pragma unroll
    for (int j = 0; j < 4; j++) cnt += (uint32_t)__popcll(__ballot(e[j] < 256u));
    if (l == 0) {
      gn[w] = cnt;
      gz[w] = zg;
    }
  }
  __syncthreads();
  // step 2: wave 0 runs the ranges' summaries from the initial stack (the
  // in-use bytes ascending); gD[q] becomes range q's incoming stack and gz[q]
  // its prefix summary
  if (w == 0) {
    uint32_t e[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const uint32_t v = j * 64 + l;
      e[j] = 0x100u;
      if ((bm[v >> 5] >> (v & 31)) & 1u) {
        uint32_t pos = 0;
        for (int q = 0; q < (int)(v >> 5); q++) pos += __popc(bm[q]);
        pos += __popc(bm[v >> 5] & ((1u << (v & 31)) - 1u));
        tmp[0][pos] = v;
      }
    }
    wave_sync();
#pragma unroll
    for (int j = 0; j < 4; j++) e[j] = (uint32_t)(j * 64) + l < nu ? tmp[0][j * 64 + l] : 0x100u;
    wave_sync();
    ZSum p = zid;
    for (int q = 0; q < SW; q++) {
      uint32_t dx[4];
      const uint32_t nd = gn[q];
#pragma unroll
      for (int j = 0; j < 4; j++) dx[j] = gD[q][j * 64 + l];
      const ZSum zq = gz[q];
      wave_sync();
#pragma unroll
      for (int j = 0; j < 4; j++) gD[q][j * 64 + l] = (uint8_t)(e[j] & 255u);
      if (l == 0) gz[q] = p;
      stack_front(e, dx, nd, mem[0], tmp[0]);
      p = zcombine(p, zq);
    }
    // flush of the last zero run, end of block (no symbols for an empty block)
    if (l == 0) nsyms[b] = nc ? zs_out(p) + run_digits(zs_carry(p)) + 1u : 0u;
  }
  __syncthreads();
  // step 3: every wave walks its range from its incoming stack and summary
  {
    uint32_t e[4];
#pragma unroll
    for (int j = 0; j < 4; j++) e[j] = (uint32_t)(j * 64) + l < nu ? (uint32_t)gD[w][j * 64 + l] : 0x100u;
    ZSum p = gz[w];
    uint32_t dn[4] = {0, 0, 0, 0}, ndn = 0;
    ZSum zn = zid;
    if (r0 < r1) load_d(r0, dn, ndn, zn);
    for (uint32_t c = r0; c < r1; c++) {
      uint32_t dx[4] = {dn[0], dn[1], dn[2], dn[3]};
      const uint32_t nd = ndn;
      const ZSum z = zn;
      if (c + 1 < r1) load_d(c + 1, dn, ndn, zn);
#pragma unroll
      for (int j = 0; j < 4; j++) chunk_list[(size_t)c * 256 + j * 64 + l] = (uint8_t)(e[j] & 255u);
      if (l == 0) {
        chunk_carry[c] = zs_carry(p);
        chunk_out[c] = zs_out(p);
      }
      stack_front(e, dx, nd, mem[w], tmp[w]);
      p = zcombine(p, z);
    }
  }
}

// Stack column j of the wave: slot j*64 + lane.  A DPP wave_shr:1 moves every
// lane's value one lane up; lane 0 keeps `into`.
__device__ __forceinline__ uint32_t wave_shift_in(uint32_t into, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)into, (int)v, 0x138, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t first_lane(uint64_t m) { return (uint32_t)(__ffsll((long long)m) - 1); }

// One wave per chunk: MTF from the chunk's incoming stack, RUNA/RUNB.
//
// Rows whose MTF index is 0 (the byte repeats the previous one) are found 64
// at a time by one ballot.  A batch of 64 rows with few nonzero indices runs
// the serial step for those rows only: search the stack columns that can hold
// in-use bytes, shift.  A batch with many runs the batched step, which has
// no serial chain: for row l holding byte x,
//   * if x occurred earlier in the batch (last at lane p), its index is the
//     number of distinct bytes in lanes p+1..l-1 = lanes k < l whose next
//     occurrence is at or after l, i.e. lanes below l minus the "previous
//     occurrence" lanes of rows below l (an exclusive prefix-OR);
//   * else its index is D + R(x) - #{first-occurrence lanes k < l with
//     R(x_k) < R(x)}, with R the position in the stack before the batch and D
//     the number of distinct bytes in lanes below l;
// and the stack becomes [the batch's bytes by last occurrence, latest first]
// followed by the rest in their old order.  Emitted symbols of the serial
// path collect in one register (stored 64 at a time); the batched path
// stores its symbols directly at their prefix-sum offsets.
template <int NCOL>
__device__ void mtf_emit_chunk(const uint8_t* __restrict__ L, const ChunkGeom& g, uint32_t nu, const uint8_t* lst,
                               uint32_t zrun, uint64_t obase, uint16_t* __restrict__ syms, uint32_t* fq,
                               uint32_t* posof, uint32_t* nstk, uint32_t* inb, uint32_t* __restrict__ err) {
  constexpr int BATCHED_MIN = 16;  // nonzero rows from which a batch takes the batched step
  const uint32_t l = lane();
  const uint64_t lt = lanemask_lt();
  uint32_t e0 = l < nu ? lst[l] : 0x100u;
  uint32_t e1 = (NCOL > 1 && 64 + l < nu) ? lst[64 + l] : 0x100u;
  uint32_t e2 = (NCOL > 2 && 128 + l < nu) ? lst[128 + l] : 0x100u;
  uint32_t e3 = (NCOL > 3 && 192 + l < nu) ? lst[192 + l] : 0x100u;
  uint32_t wc = 0;    // symbols emitted so far by this chunk
  uint32_t ob = 0;    // symbols [ob, wc) are pending in outv (lane i = symbol ob + i)
  uint32_t outv = 0;
  // the byte before the chunk is the front of its incoming stack (at the
  // block start: the smallest in-use byte, which MTF index 0 refers to)
  uint32_t prev = (uint32_t)__builtin_amdgcn_readlane((int)e0, 0);
  auto flush = [&]() {
    const uint32_t n = wc - ob;
    if (n && l < n) {
      syms[obase + ob + l] = (uint16_t)outv;
      atomicAdd(&fq[outv], 1u);
    }
    ob = wc;
  };
  auto emit = [&](uint32_t sym) {
    outv = (l == wc - ob) ? sym : outv;
    wc++;
    if (wc - ob == 64) flush();
  };
  auto emit_run = [&](uint32_t r) {
    while (r) {
      if (r & 1u) {
        emit(0);
        r = (r - 1) >> 1;
      } else {
        emit(1);
        r = (r - 2) >> 1;
      }
    }
  };
  uint32_t nxt = (g.lo + l < g.hi) ? (uint32_t)L[g.lo + l] : 0x1FFu;
  for (uint32_t base = g.lo; base < g.hi; base += 64) {
    const uint32_t cnt = min(64u, g.hi - base);
    const bool valid = l < cnt;
    const uint32_t mine = valid ? nxt : 0x1FFu;
    nxt = (base + 64 + l < g.hi) ? (uint32_t)L[base + 64 + l] : 0x1FFu;  // prefetch the next batch
    const uint32_t before = wave_shift_in(prev, mine);
    uint64_t nz = __ballot(valid && mine != before);
    if (__popcll(nz) < BATCHED_MIN) {
      // ---------------- serial step for the few nonzero rows
      int last = -1;
      while (nz) {
        const int i = (int)first_lane(nz);
        nz &= nz - 1;
        zrun += (uint32_t)(i - last - 1);
        last = i;
        const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)mine, i);
        uint32_t pos;
        const uint64_t m0 = __ballot(e0 == x);
        if (m0) {
          pos = first_lane(m0);
        } else {
          const uint64_t m1 = NCOL > 1 ? __ballot(e1 == x) : 0ull;
          if (m1) {
            pos = 64u + first_lane(m1);
          } else {
            const uint64_t m2 = NCOL > 2 ? __ballot(e2 == x) : 0ull;
            if (m2) {
              pos = 128u + first_lane(m2);
            } else {
              const uint64_t m3 = NCOL > 3 ? __ballot(e3 == x) : 0ull;
              if (m3) {
                pos = 192u + first_lane(m3);
              } else {  // byte missing from the stack: inconsistent in-use map
                if (l == 0) atomicOr(err, 1u);
                pos = 1;
              }
            }
          }
        }
        emit_run(zrun);
        zrun = 0;
        emit(pos + 1);
        // slots 1..pos take the slot above them, slot 0 takes x
        uint32_t old = e0;
        uint32_t sh = wave_shift_in(x, old);
        e0 = (l <= pos) ? sh : old;
        if (NCOL > 1 && pos >= 64) {
          uint32_t into = (uint32_t)__builtin_amdgcn_readlane((int)old, 63);
          old = e1;
          sh = wave_shift_in(into, old);
          e1 = (64 + l <= pos) ? sh : old;
          if (NCOL > 2 && pos >= 128) {
            into = (uint32_t)__builtin_amdgcn_readlane((int)old, 63);
            old = e2;
            sh = wave_shift_in(into, old);
            e2 = (128 + l <= pos) ? sh : old;
            if (NCOL > 3 && pos >= 192) {
              into = (uint32_t)__builtin_amdgcn_readlane((int)old, 63);
              old = e3;
              sh = wave_shift_in(into, old);
              e3 = (192 + l <= pos) ? sh : old;
            }
          }
        }
      }
      zrun += (uint32_t)((int)cnt - 1 - last);
    } else {
      // ---------------- batched step
      flush();
      if (e0 < 256u) posof[e0] = l;
      if (NCOL > 1 && e1 < 256u) posof[e1] = 64u + l;
      if (NCOL > 2 && e2 < 256u) posof[e2] = 128u + l;
      if (NCOL > 3 && e3 < 256u) posof[e3] = 192u + l;
      __syncthreads();
      const uint64_t vmask = __ballot(valid);
      const uint32_t R = valid ? posof[mine] : 0x3FFu;
      const uint64_t peers = match_digit8(mine & 255u, vmask);
      const uint64_t pm = peers & lt;
      const int p = pm ? 63 - (int)__clzll((long long)pm) : -1;          // previous occurrence
      const uint64_t nm = peers & ~lt & ~(1ull << l);
      const bool is_last = valid && nm == 0;                              // no later occurrence
      const uint64_t first_m = __ballot(valid && p < 0);
      const uint64_t last_m = __ballot(is_last);
      // N = lanes k that are the previous occurrence of some lane m < l
      const uint64_t incl = wave_incl_or((valid && p >= 0) ? (1ull << p) : 0ull);
      const uint64_t N = wave_shr1(uint64_t(0), incl);
      // below = #{first-occurrence lanes k < l with R_k < R_l}, one ballot
      // per bit of R from the top: at bit b, lanes that agree with R_l above
      // b and have a 0 where R_l has a 1 are smaller
      uint32_t below = 0;
      {
        uint64_t eq = first_m & lt;
#pragma unroll
        for (int b = 7; b >= 0; b--) {
          const bool mb = (R >> b) & 1u;
          const uint64_t B = __ballot(mb);
          if (mb) below += (uint32_t)__popcll(eq & ~B);
          eq &= mb ? B : ~B;
        }
      }
      uint32_t idx;
      if (p >= 0) {
        const uint64_t upto_p = (p >= 63) ? ~0ull : ((2ull << p) - 1ull);
        idx = (uint32_t)__popcll(lt & ~N & ~upto_p);
      } else {
        idx = (uint32_t)__popcll(first_m & lt) + R - below;
      }
      if (!valid) idx = 0;
      // RUNA/RUNB: a nonzero row emits the digits of the zero run before it
      const uint64_t nzm = __ballot(valid && idx != 0);
      const uint64_t pz = nzm & lt;
      const int pnz = pz ? 63 - (int)__clzll((long long)pz) : -1;
      const bool isnz = (nzm >> l) & 1ull;
      uint32_t r = (uint32_t)((int)l - pnz - 1) + (pnz < 0 ? zrun : 0u);
      const uint32_t ndig = isnz ? run_digits(r) : 0u;
      const uint32_t cnt_e = isnz ? ndig + 1u : 0u;
      const uint32_t inc = wave_incl_sum(cnt_e);
      const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
      if (isnz) {
        uint64_t o = obase + wc + inc - cnt_e;
        while (r) {
          if (r & 1u) {
            syms[o++] = 0;
            atomicAdd(&fq[0], 1u);
            r = (r - 1) >> 1;
          } else {
            syms[o++] = 1;
            atomicAdd(&fq[1], 1u);
            r = (r - 2) >> 1;
          }
        }
        syms[o] = (uint16_t)(idx + 1);
        atomicAdd(&fq[idx + 1], 1u);
      }
      wc += total;
      ob = wc;
      const int lnz = nzm ? 63 - (int)__clzll((long long)nzm) : -1;
      zrun = (lnz < 0) ? zrun + cnt : (uint32_t)((int)cnt - 1 - lnz);
      // new stack: batch bytes by last occurrence, then the rest in order
      const uint32_t nd = (uint32_t)__popcll(first_m);
      if (valid && p < 0) inb[mine] = 1u;
      __syncthreads();
      if (is_last) nstk[__popcll(last_m & ~(lt | (1ull << l)))] = mine;
      uint32_t seen = 0;
      // the columns' membership reads first, all together (they precede
      // the nstk writes, which the compiler keeps in order with them)
      const uint32_t ib0 = inb[e0 & 255u];
      const uint32_t ib1 = NCOL > 1 ? inb[e1 & 255u] : 0u;
      const uint32_t ib2 = NCOL > 2 ? inb[e2 & 255u] : 0u;
      const uint32_t ib3 = NCOL > 3 ? inb[e3 & 255u] : 0u;
#define BZG_RESTACK(ej, ibj, J)                                                \
  {                                                                            \
    const bool in_b = ((ej) < 256u) & ((ibj) != 0u);                           \
    const uint64_t cm = __ballot(in_b);                                        \
    if (!in_b) nstk[nd + (J) * 64u + l - (seen + (uint32_t)__popcll(cm & lt))] = (ej); \
    seen += (uint32_t)__popcll(cm);                                            \
  }
      BZG_RESTACK(e0, ib0, 0)
      if (NCOL > 1) BZG_RESTACK(e1, ib1, 1)
      if (NCOL > 2) BZG_RESTACK(e2, ib2, 2)
      if (NCOL > 3) BZG_RESTACK(e3, ib3, 3)
#undef BZG_RESTACK
      __syncthreads();
      e0 = nstk[l];
      if (NCOL > 1) e1 = nstk[64 + l];
      if (NCOL > 2) e2 = nstk[128 + l];
      if (NCOL > 3) e3 = nstk[192 + l];
      if (valid && p < 0) inb[mine] = 0u;
      __syncthreads();
    }
    prev = (uint32_t)__builtin_amdgcn_readlane((int)mine, (int)cnt - 1);
  }
  if (g.last) {
    emit_run(zrun);
    emit(nu + 1);
  }
  flush();
}

__device__ void mtf_emit_one(uint32_t c, const uint8_t* __restrict__ L, const uint32_t* chunk_blk,
                             const uint32_t* blk_chunk0, const uint32_t* off, const uint32_t* __restrict__ inuse,
                             const uint8_t* __restrict__ chunk_list, const uint32_t* __restrict__ chunk_carry,
                             const uint32_t* __restrict__ chunk_out, const uint64_t* __restrict__ sym_base,
                             uint16_t* __restrict__ syms, uint32_t* __restrict__ freq, uint32_t* __restrict__ err,
                             uint32_t ch) {
  __shared__ uint32_t fq[MAXA];
  __shared__ uint32_t posof[256], nstk[256], inb[256];
  const uint32_t l = lane();
  ChunkGeom g = chunk_geom(c, chunk_blk, blk_chunk0, off, ch);
  uint32_t nu = 0;
  for (int j = 0; j < 8; j++) nu += __popc(inuse[g.b * 8 + j]);
  for (uint32_t i = l; i < MAXA; i += 64) fq[i] = 0;
  for (uint32_t i = l; i < 256; i += 64) inb[i] = 0;
  __syncthreads();
  const uint8_t* lst = chunk_list + (size_t)c * 256;
  const uint32_t zrun = chunk_carry[c];
  const uint64_t obase = sym_base[g.b] + chunk_out[c];
  if (nu <= 64) mtf_emit_chunk<1>(L, g, nu, lst, zrun, obase, syms, fq, posof, nstk, inb, err);
  else if (nu <= 128) mtf_emit_chunk<2>(L, g, nu, lst, zrun, obase, syms, fq, posof, nstk, inb, err);
  else if (nu <= 192) mtf_emit_chunk<3>(L, g, nu, lst, zrun, obase, syms, fq, posof, nstk, inb, err);
  else mtf_emit_chunk<4>(L, g, nu, lst, zrun, obase, syms, fq, posof, nstk, inb, err);
  __syncthreads();
  for (uint32_t i = l; i < nu + 2; i += 64)
    if (fq[i]) atomicAdd(&freq[(size_t)g.b * MAXA + i], fq[i]);
}

// One wave per chunk, persistent over the *n_chunks chunks (at most cap).
__global__ __launch_bounds__(BZG_WAVE) void k_mtf_emit(const uint8_t* __restrict__ L, const uint32_t* chunk_blk,
                                                       const uint32_t* blk_chunk0, const uint32_t* off,
                                                       const uint32_t* __restrict__ inuse,
                                                       const uint8_t* __restrict__ chunk_list,
                                                       const uint32_t* __restrict__ chunk_carry,
                                                       const uint32_t* __restrict__ chunk_out,
                                                       const uint64_t* __restrict__ sym_base, uint16_t* __restrict__ syms,
                                                       uint32_t* __restrict__ freq, uint32_t* __restrict__ err,
                                                       uint32_t ch, const uint32_t* __restrict__ n_chunks, uint32_t cap) {
  for (TileLoop it = tile_loop(min(*n_chunks, cap)); it.t < it.end; it.t += it.step) {
    mtf_emit_one(it.t, L, chunk_blk, blk_chunk0, off, inuse, chunk_list, chunk_carry, chunk_out, sym_base, syms, freq,
                 err, ch);
    __syncthreads();
  }
}

// ------------------------------------------------------------- host side

// Chunk rows for a call of at most `rows` rows in `nb` blocks.
uint32_t mtf_chunk_rows(uint64_t rows, uint32_t nb) {
  if (g_tune && (g_tune->mtf_chunk == MTF_CHUNK || g_tune->mtf_chunk == MTF_CHUNK_SMALL)) return g_tune->mtf_chunk;
  return (rows / MTF_CHUNK + nb) < MTF_FEW_CHUNKS ? MTF_CHUNK_SMALL : MTF_CHUNK;
}
static uint64_t chunk_bound(uint64_t rows, uint32_t nb, uint32_t ch) { return rows / ch + nb + 1; }

size_t mtf_workspace_bytes(uint64_t rows, uint32_t nb) {
  const uint32_t ch = mtf_chunk_rows(rows, nb);
  const size_t nc = chunk_bound(rows, nb, ch);
  return 9 * 256 + (nc + 1) * (4 + 256 + 4 + sizeof(ZSum) + 256 + 4 + 4 + 32) + (nb + 1) * 4 + 4096;
}

// MTF and RUNA/RUNB of blocks [off[b], off[b+1]) of L (nb blocks, some
// possibly empty; at most `rows` rows), chunked: chunk_blk/blk_chunk0 give
// the chunk map (*n_chunks chunks, built on the device from the same
// chunk size mtf_chunk_rows(rows, nb)).
hipError_t mtf_run(const uint8_t* L, const uint32_t* d_off, uint32_t nb, uint64_t rows, const uint32_t* chunk_blk,
                   const uint32_t* blk_chunk0, const uint32_t* n_chunks, void* ws, size_t ws_bytes, uint16_t* syms,
                   const uint64_t* d_sym_base, uint32_t* nsyms, uint32_t* inuse, uint32_t* freq, uint32_t* err,
                   std::string& emsg, hipStream_t st) {
  const uint32_t ch = mtf_chunk_rows(rows, nb);
  const uint32_t nc = (uint32_t)chunk_bound(rows, nb, ch);
  Bump bump;
  bump.base = (char*)ws;
  bump.cap = ws_bytes;
  uint8_t* d_D = bump.take<uint8_t>((size_t)nc * 256);
  uint32_t* d_nD = bump.take<uint32_t>(nc + 1);
  ZSum* d_sum = bump.take<ZSum>(nc + 1);
  uint8_t* d_list = bump.take<uint8_t>((size_t)nc * 256);
  uint32_t* d_carry = bump.take<uint32_t>(nc + 1);
  uint32_t* d_out = bump.take<uint32_t>(nc + 1);
  uint32_t* d_cin = bump.take<uint32_t>((size_t)nc * 8 + 8);
  if (bump.used > ws_bytes) {
    emsg = "mtf workspace too small";
    return hipErrorInvalidValue;
  }
  if (nb == 0) return hipSuccess;
  const uint32_t gs = persist_grid(nc, ONE_TILE_EACH), ge = persist_grid(nc, ONE_TILE_EACH);
  {
    ProfScope ps("mtf_state", st, 0, d_off + nb, 1.0, n_chunks, 256.0);
    if (ch == MTF_CHUNK)
      hipLaunchKernelGGL(k_mtf_state<MTF_CHUNK>, dim3(gs), dim3(NT), 0, st, L, chunk_blk, blk_chunk0, d_off, d_cin, d_D,
                         d_nD, d_sum, n_chunks, nc);
    else
      hipLaunchKernelGGL(k_mtf_state<MTF_CHUNK_SMALL>, dim3(gs), dim3(NT), 0, st, L, chunk_blk, blk_chunk0, d_off,
                         d_cin, d_D, d_nD, d_sum, n_chunks, nc);
  }
  {
    ProfScope ps("mtf_scan", st, 0, n_chunks, 512.0);
    if (nc >= SCAN_LARGE_CHUNKS * nb)
      hipLaunchKernelGGL(k_mtf_scan<SCAN_WAVES_LARGE>, dim3(nb), dim3(SCAN_WAVES_LARGE * BZG_WAVE), 0, st, blk_chunk0,
                         d_cin, inuse, freq, err, L, d_off, d_D, d_nD, d_sum, d_list, d_carry, d_out, nsyms);
    else
      hipLaunchKernelGGL(k_mtf_scan<SCAN_WAVES>, dim3(nb), dim3(SCAN_WAVES * BZG_WAVE), 0, st, blk_chunk0, d_cin,
                         inuse, freq, err, L, d_off, d_D, d_nD, d_sum, d_list, d_carry, d_out, nsyms);
  }
  {
    ProfScope ps("mtf_emit", st, 0, d_off + nb, 3.0);  // read L, write at most one 2-byte symbol per row
    hipLaunchKernelGGL(k_mtf_emit, dim3(ge), dim3(BZG_WAVE), 0, st, L, chunk_blk, blk_chunk0, d_off, inuse, d_list,
                       d_carry, d_out, d_sym_base, syms, freq, err, ch, n_chunks, nc);
  }
  return hipGetLastError();
}

}  // namespace bzg
