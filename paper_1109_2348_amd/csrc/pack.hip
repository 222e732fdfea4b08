// Variable-length packing and stream assembly (Sec. 3.4, Figure 3: look up
// every symbol's code and length, take the prefix sum of the lengths as bit
// offsets, write every code at its offset).
//
// Bits are written MSB-first straight into their final place in the output
// stream, so blocks need no later bit-shifting copy: block bit offsets are a
// prefix sum of block sizes, group offsets a prefix sum of group sizes, symbol
// offsets a prefix sum inside a tile.  A tile assembles its words in LDS;
// words wholly inside the tile are stored, the two edge words are OR-ed in
// atomically (the buffer is zeroed first).  Words hold stream bits in
// big-endian order and are byte-swapped on store.
#include <climits>

#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace bzg {

__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

constexpr uint32_t SEL_CHUNK = 8192;                         // selectors staged in LDS at a time
constexpr uint32_t SEL_WORDS = (SEL_CHUNK * MAXG + 31) / 32 + 2;  // their unary codes, 32-bit words

// OR the low n (<= 32) bits of v into the stream at bit position pos.
__device__ __forceinline__ void put_bits(uint32_t* words, uint64_t pos, uint32_t v, uint32_t n) {
  if (n == 0) return;
  v &= (n == 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
  uint64_t wi = pos >> 5;
  uint32_t o = (uint32_t)(pos & 31);
  if (o + n <= 32) {
    atomicOr(&words[wi], bswap32(v << (32 - o - n)));
  } else {
    uint32_t spill = o + n - 32;
    atomicOr(&words[wi], bswap32(v >> spill));
    atomicOr(&words[wi + 1], bswap32(v << (32 - spill)));
  }
}

__device__ __forceinline__ void put_bits64(uint32_t* words, uint64_t pos, uint64_t v, uint32_t n) {
  if (n > 32) {
    put_bits(words, pos, (uint32_t)(v >> 32), n - 32);
    put_bits(words, pos + (n - 32), (uint32_t)v, 32);
  } else {
    put_bits(words, pos, (uint32_t)v, n);
  }
}

// Block layout: bit offset of every block and each stream's end.  One
// workgroup per stream.  mode 0: one bzip2 stream per request r, made of
// blocks [rb[r], rb[r+1]) and written from byte rout[r] of the output; blocks
// follow the 32-bit stream header and carry the 105-bit block header; empty
// blocks (no tables) take no bits and do not count.  info[2r] = the stream's
// length in bits (with the end-of-stream marker and combined CRC),
// info[2r+1] = the combined CRC; out_bytes[r] = its length in bytes; a stream
// that does not fit its range [rout[r], rout[r+1]) (rounded up to 4 bytes)
// sets ERR_CAPACITY and the skip flag (*skip) that the packing kernels test.
// n_blocks (optional) gets the blocks of stream 0.  mode 1: bodies only,
// block b at body_byte[b] * 8 (rb, rout unused, one workgroup): nbits[b]
// = its bits, checked against body_byte[b + 1].
__global__ __launch_bounds__(NT) void k_layout(uint32_t nb, const BlockTables* __restrict__ tabs, int mode,
                                               const uint32_t* __restrict__ rb, const uint64_t* __restrict__ rout,
                                               const uint64_t* __restrict__ body_byte, uint64_t* __restrict__ blk_bit,
                                               const uint32_t* __restrict__ crc, uint64_t* __restrict__ info,
                                               uint64_t* __restrict__ out_bytes, uint32_t* __restrict__ n_blocks,
                                               const uint32_t* __restrict__ slot_base, uint32_t* __restrict__ skip,
                                               uint32_t* __restrict__ err) {
  __shared__ uint64_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t sh32[NT / BZG_WAVE + 1];
  __shared__ uint32_t shx[NT / BZG_WAVE];
  const uint32_t r = blockIdx.x;
  // rb counts input blocks; slot_base turns them into slots (blocks after cutting)
  const uint32_t b0 = mode == 0 ? slot_base[rb[r]] : 0u, b1 = mode == 0 ? slot_base[rb[r + 1]] : nb;
  const uint64_t base = mode == 0 ? rout[r] * 8 : 0;
  // blocks of the stream that are not empty, counted first: the combined
  // CRC rotates each block's CRC once per non-empty block after it
  uint32_t cnt = 0;
  for (uint32_t c = b0 + threadIdx.x; c < b1; c += NT) cnt += tabs[c].G ? 1u : 0u;
  const uint32_t nne = block_sum<uint32_t, NT>(cnt, sh32);
  uint64_t carry = 32;
  uint32_t comb = 0, seen = 0, over = 0;
  for (uint32_t c = b0; c < b1; c += NT) {
    uint32_t b = c + threadIdx.x;
    uint64_t sz = 0;
    uint32_t ne = 0;
    if (b < b1 && tabs[b].G) {
      sz = (mode == 0 ? 105u : 0u) + tabs[b].hdr_bits + tabs[b].data_bits;
      ne = 1;
    }
    uint64_t tot;
    uint64_t ex = block_excl_sum<uint64_t, NT>(sz, sh, &tot);
    uint32_t net;
    const uint32_t nex = block_excl_sum<uint32_t, NT>(ne, sh32, &net);
    if (b < b1) {
      blk_bit[b] = mode == 0 ? base + carry + ex : body_byte[b] * 8;
      if (mode == 0 && ne) {
        const uint32_t k = (nne - 1 - (seen + nex)) & 31u, v = crc[b];
        comb ^= k ? (v << k) | (v >> (32 - k)) : v;
      }
      if (mode == 1) {
        const uint64_t bits = (uint64_t)tabs[b].hdr_bits + tabs[b].data_bits;
        info[b] = bits;
        if (bits > (body_byte[b + 1] - body_byte[b]) * 8) over = 1;
      }
    }
    carry += tot;
    seen += net;
  }
  comb = wave_xor(comb);
  if (lane() == 0) shx[threadIdx.x / BZG_WAVE] = comb;
  over = block_sum<uint32_t, NT>(over, sh32);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / BZG_WAVE; w++) comb ^= shx[w];
    if (mode == 0) {
      const uint64_t bits = carry + 80;  // stream bits incl. end-of-stream marker and CRC
      info[2 * r] = bits;
      info[2 * r + 1] = comb;
      out_bytes[r] = (bits + 7) / 8;
      if (n_blocks && r == 0) *n_blocks = nne;
      over = (bits + 31) / 32 * 4 > rout[r + 1] - rout[r];
    }
    if (over) {
      atomicOr(skip, 1u);
      atomicOr(err, ERR_CAPACITY);
    }
  }
}

// Zero the words each stream will occupy (bits are OR-ed in afterwards).
// Grid (x, streams); a plain fill kernel, so the call stays capturable.
__global__ __launch_bounds__(NT) void k_zero_streams(const uint64_t* __restrict__ rout,
                                                     const uint64_t* __restrict__ info, uint32_t* __restrict__ words,
                                                     const uint32_t* __restrict__ skip) {
  if (*skip) return;
  const uint32_t r = blockIdx.y;
  const uint64_t w0 = rout[r] / 4, nw = (info[2 * r] + 31) / 32;
  for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < nw; i += (uint64_t)gridDim.x * NT) words[w0 + i] = 0;
}

// Block header and body head: [magic, CRC, rand bit, origPtr,] symbol map,
// table count, selector count, unary MTF'd selectors, delta-coded lengths.
__global__ __launch_bounds__(NT) void k_pack_header(const BlockTables* __restrict__ tabs, int mode,
                                                    const uint64_t* __restrict__ blk_bit,
                                                    const uint32_t* __restrict__ crc,
                                                    const uint32_t* __restrict__ primary,
                                                    const uint32_t* __restrict__ inuse,
                                                    const uint64_t* __restrict__ sel_base,
                                                    const uint8_t* __restrict__ selmtf, uint32_t* __restrict__ words,
                                                    const uint32_t* __restrict__ skip) {
  __shared__ uint64_t sh[NT / BZG_WAVE + 1];
  const uint32_t b = blockIdx.x;
  const BlockTables* T = &tabs[b];
  const uint32_t G = T->G, nsel = T->nsel, a = T->alpha;
  if (*skip || G == 0) return;  // output too small, or an empty block
  uint64_t pos = blk_bit[b];
  if (mode == 0) {
    if (threadIdx.x == 0) {
      put_bits64(words, pos, 0x314159265359ull, 48);
      put_bits(words, pos + 48, crc[b], 32);
      put_bits(words, pos + 81, primary[b], 24);  // bit 80 is the (zero) randomised flag
    }
    pos += 105;
  }
  uint32_t bm[8];
  uint32_t ranges = 0, nr = 0;
  for (int j = 0; j < 8; j++) {
    bm[j] = inuse[b * 8 + j];
    for (int hlf = 0; hlf < 2; hlf++) {
      uint32_t r = 2 * j + hlf;
      if ((bm[j] >> (16 * hlf)) & 0xFFFFu) {
        ranges |= 1u << (15 - r);
        nr++;
      }
    }
  }
  if (threadIdx.x == 0) put_bits(words, pos, ranges, 16);
  pos += 16;
  if (threadIdx.x < 16 && ((ranges >> (15 - threadIdx.x)) & 1u)) {
    uint32_t r = threadIdx.x;
    uint32_t k = __popc(ranges >> (16 - r)) ;  // used ranges before r
    if (r == 0) k = 0;
    uint32_t half = (bm[r >> 1] >> (16 * (r & 1))) & 0xFFFFu;
    uint32_t v = 0;  // bit j (MSB first) = byte 16r + j in use
    for (int j = 0; j < 16; j++) v |= ((half >> j) & 1u) << (15 - j);
    put_bits(words, pos + 16 * k, v, 16);
  }
  pos += 16 * nr;
  if (threadIdx.x == 0) {
    put_bits(words, pos, G, 3);
    put_bits(words, pos + 3, nsel, 15);
  }
  pos += 18;
  // selectors in unary (idx ones, then a zero), SEL_CHUNK at a time: staged
  // in LDS, coded into LDS words (thread-contiguous ranges), written out
  // coalesced; only a chunk's first and last words are shared with others
  const uint8_t* M = selmtf + sel_base[b];
  __shared__ uint8_t sM[SEL_CHUNK];
  __shared__ uint32_t sw[SEL_WORDS];
  for (uint32_t c0 = 0; c0 < nsel; c0 += SEL_CHUNK) {
    const uint32_t cn = min(SEL_CHUNK, nsel - c0);
    __syncthreads();
    stage_to_lds<NT, 8>(sM, M + c0, cn);
    for (uint32_t i = threadIdx.x; i < SEL_WORDS; i += NT) sw[i] = 0;
    __syncthreads();
    const uint32_t per = (cn + NT - 1) / NT;
    const uint32_t g0 = min(threadIdx.x * per, cn), g1 = min(g0 + per, cn);
    uint64_t mine = 0;
    for (uint32_t g = g0; g < g1; g++) mine += sM[g] + 1u;
    uint64_t tot;
    const uint32_t off = (uint32_t)(pos & 31);
    uint32_t p = off + (uint32_t)block_excl_sum<uint64_t, NT>(mine, sh, &tot);
    for (uint32_t g = g0; g < g1; g++) {
      const uint32_t n = sM[g] + 1u, v = (1u << n) - 2u, o = p & 31u;  // n <= MAXG
      if (o + n <= 32) {
        atomicOr(&sw[p >> 5], v << (32 - o - n));
      } else {
        atomicOr(&sw[p >> 5], v >> (o + n - 32));
        atomicOr(&sw[(p >> 5) + 1], v << (64 - o - n));
      }
      p += n;
    }
    __syncthreads();
    const uint32_t nw = (uint32_t)((off + tot + 31) / 32);
    const uint64_t W0 = pos >> 5;
    for (uint32_t i = threadIdx.x; i < nw; i += NT) {
      const uint32_t v = sw[i];
      if (i == 0 || i + 1 == nw) {
        if (v) atomicOr(&words[W0 + i], bswap32(v));
      } else {
        words[W0 + i] = bswap32(v);
      }
    }
    pos += tot;
  }
  // code lengths, one table after another: each table's 5-bit start, then
  // per symbol the delta code.  Lengths staged in LDS; one workgroup scan of
  // all tables' bit counts (thread-contiguous items: table i / a, symbol i % a)
  __shared__ uint8_t slen[MAXG][MAXA];
  __syncthreads();
  stage_to_lds<NT, 8>(&slen[0][0], &T->len[0][0], G * MAXA);
  __syncthreads();
  constexpr uint32_t PI = (MAXG * MAXA + NT - 1) / NT;  // items per thread (<= 7)
  const uint32_t nit = G * a;
  const uint32_t i0 = min(threadIdx.x * PI, nit), i1 = min(i0 + PI, nit);
  uint64_t mine = 0;
  for (uint32_t i = i0; i < i1; i++) {
    const uint32_t t = i / a, v = i % a;
    const int d = (int)slen[t][v] - (int)slen[t][v ? v - 1 : 0];
    mine += (v == 0 ? 5u : 0u) + 2u * (uint32_t)(d < 0 ? -d : d) + 1u;
  }
  uint64_t tt;
  uint64_t q = pos + block_excl_sum<uint64_t, NT>(mine, sh, &tt);
  for (uint32_t i = i0; i < i1; i++) {
    const uint32_t t = i / a, v = i % a;
    if (v == 0) {
      put_bits(words, q, slen[t][0], 5);
      q += 5;
    }
    const int d = (int)slen[t][v] - (int)slen[t][v ? v - 1 : 0];
    const uint32_t ad = (uint32_t)(d < 0 ? -d : d), n = 2u * ad + 1u;
    uint64_t code = 0;
    const uint32_t step = d < 0 ? 3u : 2u;
    for (uint32_t k = 0; k < ad; k++) code = (code << 2) | step;
    code <<= 1;
    put_bits64(words, q, code, n);
    q += n;
  }
}

// Data codes: tile = PACK_GROUPS selector groups of one block.
__device__ void pack_data_tile(uint32_t j, const BlockTables* __restrict__ tabs, int mode,
                                                  const uint32_t* __restrict__ tile_blk,
                                                  const uint32_t* __restrict__ blk_tile0,
                                                  const uint64_t* __restrict__ blk_bit,
                                                  const uint16_t* __restrict__ syms,
                                                  const uint64_t* __restrict__ sym_base,
                                                  const uint32_t* __restrict__ nsyms,
                                                  const uint64_t* __restrict__ sel_base,
                                                  const uint8_t* __restrict__ sel,
                                                  const uint64_t* __restrict__ gofs, uint32_t* __restrict__ words) {
  constexpr uint32_t MAXSYM = PACK_GROUPS * GROUP;               // 3200
  constexpr uint32_t PER = (MAXSYM + NT - 1) / NT;               // 13
  constexpr uint32_t WCAP = (MAXSYM * MAXLEN) / 32 + 4;          // staging words
  __shared__ uint32_t stage[WCAP];
  __shared__ uint8_t slen[MAXG][MAXA];
  __shared__ uint32_t scode[MAXG][MAXA];
  __shared__ uint64_t sh[NT / BZG_WAVE + 1];
  const uint32_t b = tile_blk[j];
  const BlockTables* T = &tabs[b];
  const uint32_t nsel = T->nsel, G = T->G;
  const uint32_t g0 = (j - blk_tile0[b]) * PACK_GROUPS;
  if (g0 >= nsel) return;
  const uint32_t g1 = min(g0 + PACK_GROUPS, nsel);
  const uint32_t ns = nsyms[b];
  const uint32_t s0 = g0 * GROUP, s1 = min(g1 * GROUP, ns);
  // the block's tables (whole rows of the G tables; entries past the
  // alphabet are copied but never read), loads batched and unbranched
  stage_to_lds<NT, 8>(&slen[0][0], &T->len[0][0], G * MAXA);
  stage_to_lds<NT, 8>(&scode[0][0], &T->code[0][0], G * MAXA);
  for (uint32_t i = threadIdx.x; i < WCAP; i += NT) stage[i] = 0;
  const uint64_t sb = sel_base[b];
  const uint64_t data0 = blk_bit[b] + (mode == 0 ? 105u : 0u) + T->hdr_bits;
  const uint64_t B0 = data0 + (gofs[sb + g0] - gofs[sb]);
  const uint16_t* S = syms + sym_base[b];
  // the tile's symbols and selectors into LDS: coalesced, unbranched loads
  // (clamped), all in flight together
  __shared__ uint16_t ssym[MAXSYM];
  __shared__ uint8_t ssel[PACK_GROUPS];
  const uint32_t cnt = s1 - s0;
  {
    uint32_t tmp[PER];
#pragma unroll
    for (uint32_t q = 0; q < PER; q++) tmp[q] = S[s0 + min(q * NT + threadIdx.x, cnt - 1u)];
#pragma unroll
    for (uint32_t q = 0; q < PER; q++)
      if (q * NT + threadIdx.x < cnt) ssym[q * NT + threadIdx.x] = (uint16_t)tmp[q];
    if (threadIdx.x < g1 - g0) ssel[threadIdx.x] = sel[sb + g0 + threadIdx.x];
  }
  __syncthreads();
  // blocked: PER consecutive symbols per thread; each LDS stage is read for
  // all of them before any is used (clamped positions)
  const uint32_t l0 = threadIdx.x * PER;
  uint32_t tq[PER], sq[PER], nq[PER], vq[PER];
#pragma unroll
  for (uint32_t q = 0; q < PER; q++) {
    const uint32_t l = min(l0 + q, cnt - 1u);
    tq[q] = ssel[l / GROUP];
    sq[q] = min((uint32_t)ssym[l], (uint32_t)MAXA - 1u);  // (caller-given symbols are flagged, not trusted)
  }
#pragma unroll
  for (uint32_t q = 0; q < PER; q++) {
    nq[q] = slen[tq[q]][sq[q]];
    vq[q] = scode[tq[q]][sq[q]];
  }
  uint32_t mine = 0;
#pragma unroll
  for (uint32_t q = 0; q < PER; q++) mine += l0 + q < cnt ? nq[q] : 0u;
  uint64_t tot;
  uint64_t p = (B0 & 31) + block_excl_sum<uint64_t, NT>((uint64_t)mine, sh, &tot);
#pragma unroll
  for (uint32_t q = 0; q < PER; q++) {
    const uint32_t l = l0 + q;
    if (l >= cnt) break;
    const uint32_t n = nq[q], v = vq[q];
    uint32_t wi = (uint32_t)(p >> 5), o = (uint32_t)(p & 31);
    if (o + n <= 32) {
      atomicOr(&stage[wi], v << (32 - o - n));
    } else {
      uint32_t spill = o + n - 32;
      atomicOr(&stage[wi], v >> spill);
      atomicOr(&stage[wi + 1], v << (32 - spill));
    }
    p += n;
  }
  __syncthreads();
  const uint64_t endbit = (B0 & 31) + tot;  // local bit end
  const uint32_t nw = (uint32_t)((endbit + 31) >> 5);
  const uint64_t W0 = B0 >> 5;
  for (uint32_t i = threadIdx.x; i < nw; i += NT) {
    uint32_t v = stage[i];
    if (i == 0 || i + 1 == nw) {
      if (v) atomicOr(&words[W0 + i], bswap32(v));
    } else {
      words[W0 + i] = bswap32(v);
    }
  }
}

// Persistent workgroups over the *n_tiles packing tiles (at most cap).
__global__ __launch_bounds__(NT) void k_pack_data(const BlockTables* __restrict__ tabs, int mode,
                                                  const uint32_t* __restrict__ tile_blk,
                                                  const uint32_t* __restrict__ blk_tile0,
                                                  const uint64_t* __restrict__ blk_bit,
                                                  const uint16_t* __restrict__ syms,
                                                  const uint64_t* __restrict__ sym_base,
                                                  const uint32_t* __restrict__ nsyms,
                                                  const uint64_t* __restrict__ sel_base,
                                                  const uint8_t* __restrict__ sel,
                                                  const uint64_t* __restrict__ gofs, uint32_t* __restrict__ words,
                                                  const uint32_t* __restrict__ n_tiles, uint32_t cap,
                                                  const uint32_t* __restrict__ skip) {
  if (*skip) return;
  for (TileLoop it = tile_loop(min(*n_tiles, cap)); it.t < it.end; it.t += it.step) {
    pack_data_tile(it.t, tabs, mode, tile_blk, blk_tile0, blk_bit, syms, sym_base, nsyms, sel_base, sel, gofs, words);
    __syncthreads();
  }
}

// Stream header "BZh<level>", end-of-stream marker and combined CRC of
// stream r (one workgroup per stream).
__global__ void k_stream_ends(int level, const uint64_t* __restrict__ rout, const uint64_t* __restrict__ info,
                              uint32_t* __restrict__ words, const uint32_t* __restrict__ skip) {
  if (threadIdx.x != 0 || *skip) return;
  const uint32_t r = blockIdx.x;
  const uint64_t start = rout[r] * 8, end = start + info[2 * r];
  uint32_t hdr = ((uint32_t)'B' << 24) | ((uint32_t)'Z' << 16) | ((uint32_t)'h' << 8) | (uint32_t)('0' + level);
  atomicOr(&words[start / 32], bswap32(hdr));
  put_bits64(words, end - 80, 0x177245385090ull, 48);
  put_bits(words, end - 32, (uint32_t)info[2 * r + 1], 32);
}

// Per block: byte 0 = table count, bytes 16 + 258*t + v = code lengths.
__global__ __launch_bounds__(NT) void k_tables_export(const BlockTables* __restrict__ tabs, uint8_t* __restrict__ out) {
  constexpr uint32_t STRIDE = 1568;
  const uint32_t b = blockIdx.x;
  const BlockTables* T = &tabs[b];
  for (uint32_t i = threadIdx.x; i < STRIDE; i += NT) {
    uint8_t v = 0;
    if (i == 0) {
      v = (uint8_t)T->G;
    } else if (i >= 16 && i < 16 + MAXG * MAXA) {
      uint32_t t = (i - 16) / MAXA, s = (i - 16) % MAXA;
      if (t < T->G && s < T->alpha) v = T->len[t][s];
    }
    out[(size_t)b * STRIDE + i] = v;
  }
}

// Zero the bytes [lo, hi) (4-byte aligned) unless *skip: body ranges are
// OR-ed into.
__global__ __launch_bounds__(NT) void k_zero_range(uint32_t* __restrict__ words, uint64_t nw,
                                                   const uint32_t* __restrict__ skip) {
  if (*skip) return;
  for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < nw; i += (uint64_t)gridDim.x * NT) words[i] = 0;
}

hipError_t tables_export(uint32_t nb, const void* tabs, uint8_t* out, hipStream_t st) {
  if (nb) hipLaunchKernelGGL(k_tables_export, dim3(nb), dim3(NT), 0, st, (const BlockTables*)tabs, out);
  return hipGetLastError();
}

hipError_t pack_layout(uint32_t nb, uint32_t n_req, const uint32_t* rb, const uint64_t* rout, const void* tabs,
                       int mode, const uint64_t* body_byte, uint64_t* blk_bit, const uint32_t* crc, uint64_t* info,
                       uint64_t* out_bytes, uint32_t* n_blocks, const uint32_t* slot_base, uint32_t* skip, uint32_t* err,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_layout, dim3(mode == 0 ? n_req : 1u), dim3(NT), 0, st, nb, (const BlockTables*)tabs, mode, rb,
                     rout, body_byte, blk_bit, crc, info, out_bytes, n_blocks, slot_base, skip, err);
  return hipGetLastError();
}

hipError_t zero_streams(uint32_t n_req, uint64_t max_words, const uint64_t* rout, const uint64_t* info,
                        uint32_t* words, const uint32_t* skip, hipStream_t st) {
  uint64_t gx = (max_words + NT * 8 - 1) / (NT * 8);
  gx = gx < 1 ? 1 : (gx > 1024 ? 1024 : gx);
  if (n_req) hipLaunchKernelGGL(k_zero_streams, dim3((uint32_t)gx, n_req), dim3(NT), 0, st, rout, info, words, skip);
  return hipGetLastError();
}

hipError_t zero_range(uint32_t* words, uint64_t nw, const uint32_t* skip, hipStream_t st) {
  const uint64_t g = std::min<uint64_t>((nw + NT * 4 - 1) / (NT * 4) + 1, 2048);
  if (nw) hipLaunchKernelGGL(k_zero_range, dim3((uint32_t)g), dim3(NT), 0, st, words, nw, skip);
  return hipGetLastError();
}

hipError_t pack_run(uint32_t nb, const void* tabs, int mode, const uint64_t* blk_bit, const uint32_t* crc,
                    const uint32_t* primary, const uint32_t* inuse, const uint64_t* sel_base, const uint8_t* sel,
                    const uint8_t* selmtf, const uint64_t* gofs, const uint32_t* n_tiles, uint32_t tiles_cap,
                    const uint32_t* tile_blk, const uint32_t* blk_tile0, const uint16_t* syms,
                    const uint64_t* sym_base, const uint32_t* nsyms, int level, uint32_t n_req, const uint64_t* rout,
                    const uint64_t* info, uint32_t* words, const uint32_t* skip, hipStream_t st) {
  if (nb) {
    hipLaunchKernelGGL(k_pack_header, dim3(nb), dim3(NT), 0, st, (const BlockTables*)tabs, mode, blk_bit, crc, primary,
                       inuse, sel_base, selmtf, words, skip);
    const uint32_t g = persist_grid(tiles_cap, ONE_TILE_EACH);
    hipLaunchKernelGGL(k_pack_data, dim3(g), dim3(NT), 0, st, (const BlockTables*)tabs, mode, tile_blk, blk_tile0,
                       blk_bit, syms, sym_base, nsyms, sel_base, sel, gofs, words, n_tiles, tiles_cap, skip);
  }
  if (mode == 0 && n_req)
    hipLaunchKernelGGL(k_stream_ends, dim3(n_req), dim3(64), 0, st, level, rout, info, words, skip);
  return hipGetLastError();
}

}  // namespace bzg
