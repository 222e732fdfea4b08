// Decompression of bzip2 streams on the GPU: the decoding half the paper
// discusses stage by stage --
//   variable-length decoding (Sec. 3.4: code boundaries are only known
//     serially): one wave per block finds each group's 50 code starts at
//     once by pointer doubling over the next 512 bits, the groups chained
//     in order;
//   the inverse move-to-front (Sec. 3.3) in parallel over chunks: a chunk's
//     effect on list positions is found on the identity list, the chunks'
//     permutations composed in order per block, and every symbol's byte
//     taken from its chunk's starting list, with RUNA/RUNB run lengths as
//     segmented sums;
//   the inverse BWT started from many points (Sec. 3.1): walkers start at
//     sampled rows of the last-to-first map, each stops at the next sampled
//     row, a pass along the chain of samples places every walker's piece,
//     and a second walk writes it;
//   run-length decoding in the Figure 2 pattern (Sec. 3.2): per segment, the
//     output length and outgoing state for every incoming state; a scan
//     gives each segment its state and output offset; then every segment
//     expands its runs at its offset.
// Blocks are found by a filtered search for the block and end-of-stream
// markers; the host reads back the marker list to lay the blocks out.  The
// work items of the later stages (chunks, walkers, segments) are planned on
// the device from the decoded lengths; long blocks can be decoded as a class
// of their own on a second stream.
#include "common.hpp"
#include "internal.hpp"

namespace bzg {

constexpr uint64_t MAGIC_BLOCK = 0x314159265359ull;
constexpr uint64_t MAGIC_EOS = 0x177245385090ull;
constexpr uint32_t FIND_BYTES = 16;                 // input bytes per thread of the marker search
constexpr uint32_t FIND_TILE = NT * FIND_BYTES;     // per workgroup
constexpr uint32_t DEC_LUT_BITS = 10;               // first-level decoding table
constexpr uint32_t WALK_STRIDE = 64;                // one sampled row per this many rows
constexpr uint32_t RLE_SEG = 64;                    // bytes per run-length decoding segment

// --------------------------------------------------------- marker search

// A marker that starts at bit r (0..7) of a byte covers the whole two bytes
// after it, which then hold bits 8-r .. 23-r of the magic: 8 possible 16-bit
// values per kind.  A bitmap over the top 12 bits of those values is the
// filter; positions it passes get the full 48-bit comparison.
constexpr uint32_t FIND_MAP_WORDS = 4096 / 32;
__device__ __forceinline__ void find_filter_init(uint32_t* map) {
  for (uint32_t i = threadIdx.x; i < FIND_MAP_WORDS; i += blockDim.x) map[i] = 0;
  __syncthreads();
  if (threadIdx.x < 16) {
    const uint64_t M = threadIdx.x < 8 ? MAGIC_BLOCK : MAGIC_EOS;
    const uint32_t r = threadIdx.x & 7u;
    const uint32_t v = (uint32_t)(M >> (28 + r)) & 0xFFFu;
    atomicOr(&map[v >> 5], 1u << (v & 31u));
  }
  __syncthreads();
}

// Marker candidates of the 16 bytes at b0 (bit positions 8*b0 .. +127 whose
// 48 bits lie inside the input): a bit mask per 64 positions for each kind.
__device__ __forceinline__ void find_markers(const uint8_t* __restrict__ in, uint64_t n, uint64_t b0,
                                             const uint32_t* __restrict__ map, uint64_t m[2][2]) {
  uint64_t W[3];  // the 24 bytes from b0, most significant first
  if (b0 + 24 <= n && ((uintptr_t)(in + b0) & 7u) == 0) {
#pragma unroll
    for (int w = 0; w < 3; w++) W[w] = __builtin_bswap64(((const uint64_t*)(in + b0))[w]);
  } else {
#pragma unroll
    for (int w = 0; w < 3; w++) {
      uint64_t v = 0;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const uint64_t q = b0 + 8 * w + i;
        v = (v << 8) | (q < n ? in[q] : 0u);
      }
      W[w] = v;
    }
  }
  m[0][0] = m[0][1] = m[1][0] = m[1][1] = 0;
  // bytes q+1, q+2 of the 24 loaded, for the 16 byte positions q
  uint32_t hit = 0;
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int j = q + 1;  // first of the two bytes
    const uint64_t hi = W[j / 8], lo = j / 8 + 1 < 3 ? W[j / 8 + 1] : 0ull;
    const int sh = 8 * (j % 8);  // bits of hi before byte j
    const uint64_t win = sh ? (hi << sh) | (lo >> (64 - sh)) : hi;
    const uint32_t v = (uint32_t)(win >> 52);
    hit |= ((map[v >> 5] >> (v & 31u)) & 1u) << q;
  }
  if (!hit) return;
  const uint64_t nbits = 8 * n;
  while (hit) {
    const int q = __ffs(hit) - 1;
    hit &= hit - 1;
    for (int r = 0; r < 8; r++) {
      const int p = 8 * q + r;  // bit position in the 16 bytes
      const int h = p >> 6, pp = p & 63;
      const uint64_t win = pp ? (W[h] << pp) | (W[h + 1] >> (64 - pp)) : W[h];
      const uint64_t v = win >> 16;
      const bool inside = 8 * b0 + (uint64_t)p + 48 <= nbits;
      if (inside && v == MAGIC_BLOCK) m[0][h] |= 1ull << pp;
      if (inside && v == MAGIC_EOS) m[1][h] |= 1ull << pp;
    }
  }
}

// 32 bits starting at bit q of the input (bits past the end read as 0).
__device__ __forceinline__ uint32_t bits32_at(const uint8_t* __restrict__ in, uint64_t n, uint64_t q) {
  const uint64_t b = q >> 3;
  uint64_t v = 0;
#pragma unroll
  for (int i = 0; i < 5; i++) v = (v << 8) | (b + i < n ? in[b + i] : 0u);
  return (uint32_t)(v >> (8 - (q & 7)));
}

// Pass 0: markers per workgroup tile.  Pass 1: the markers in input order,
// from the tiles' exclusive offsets: (bit position | kind << 63, the 32 bits
// after the marker | for end markers, the 4 bytes where the next stream's
// header would start << 32).
__global__ __launch_bounds__(NT) void k_find_markers(const uint8_t* __restrict__ in, uint64_t n, int pass,
                                                     uint32_t* __restrict__ tile_cnt,
                                                     const uint64_t* __restrict__ tile_off,
                                                     uint64_t* __restrict__ cand, uint64_t cand_cap) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t map[FIND_MAP_WORDS];
  find_filter_init(map);
  const uint64_t b0 = ((uint64_t)blockIdx.x * NT + threadIdx.x) * FIND_BYTES;
  uint64_t m[2][2] = {{0, 0}, {0, 0}};
  if (b0 < n) find_markers(in, n, b0, map, m);
  const uint32_t c = __popcll(m[0][0]) + __popcll(m[0][1]) + __popcll(m[1][0]) + __popcll(m[1][1]);
  uint32_t tot;
  const uint32_t ex = block_excl_sum<uint32_t, NT>(c, sh, &tot);
  if (pass == 0) {
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = tot;
    return;
  }
  if (!c) return;
  uint64_t o = tile_off[blockIdx.x] + ex;
  // in bit order: both halves, each kind merged by position
  for (int h = 0; h < 2; h++) {
    uint64_t mb = m[0][h], me = m[1][h];
    while (mb | me) {
      const int pb = mb ? __ffsll((long long)mb) - 1 : 64, pe = me ? __ffsll((long long)me) - 1 : 64;
      const bool eos = pe < pb;
      const int p = eos ? pe : pb;
      if (eos) me &= me - 1; else mb &= mb - 1;
      const uint64_t pos = 8 * b0 + 64 * h + p;
      uint64_t aux = bits32_at(in, n, pos + 48);
      if (eos) aux |= (uint64_t)bits32_at(in, n, ((pos + 80 + 7) >> 3) << 3) << 32;
      if (o < cand_cap) {
        cand[2 * o] = pos | ((uint64_t)eos << 63);
        cand[2 * o + 1] = aux;
      }
      o++;
    }
  }
}

// Exclusive offsets of n counts (one workgroup of 1024 threads); off[n] =
// the total.
__global__ __launch_bounds__(1024) void k_scan_counts(const uint32_t* __restrict__ cnt, uint32_t n,
                                                      uint64_t* __restrict__ off) {
  __shared__ uint64_t sh[1024 / BZG_WAVE + 1];
  const uint32_t per = (n + 1023) / 1024, lo = min(threadIdx.x * per, n), hi = min(lo + per, n);
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; i++) s += cnt[i];
  uint64_t tot;
  uint64_t run = block_excl_sum<uint64_t, 1024>(s, sh, &tot);
  for (uint32_t i = lo; i < hi; i++) {
    off[i] = run;
    run += cnt[i];
  }
  if (threadIdx.x == 0) off[n] = tot;
}

// ------------------------------------------------------- block decoding

// A value every lane holds alike (a table entry at a wave-uniform index),
// moved to a scalar register so that branches on it stay scalar.
template <typename T>
__device__ __forceinline__ uint32_t uni(T v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
}

// The bit stream is read through a window of 64 dwords, one per lane
// (256 bytes, most significant bit first); the next window is loaded while
// the current one is decoded, so the loop waits for memory only when it
// moves to the next window, 2048 bits after that load was issued.  Refills
// take the word from its lane with a lane read.  Past the input's end the
// last byte is read again: such bits are never part of a block.
struct BitIn {
  const uint8_t* in;
  uint64_t n;
  uint64_t wnext;  // first dword of the window being loaded
  uint32_t cur;    // this lane's dword of the current window
  uint32_t pb[4];  // this lane's bytes of the next window, as loaded
  uint32_t pos;    // next dword of the current window
  uint64_t buf;    // bits not yet used, from the top
  int nb;          // how many
  uint32_t taken;  // dwords moved into buf
  uint32_t drop;   // bits of the first dword before the start
  __device__ __forceinline__ void load_next() {
    const uint64_t q = 4 * (wnext + lane());
#pragma unroll
    for (int i = 0; i < 4; i++) pb[i] = in[min(q + i, n - 1)];
    wnext += BZG_WAVE;
  }
  __device__ __forceinline__ uint32_t joined() const { return (pb[0] << 24) | (pb[1] << 16) | (pb[2] << 8) | pb[3]; }
  // position the reader at bit `bit` of the input
  __device__ __forceinline__ void start(uint64_t bit) {
    wnext = bit >> 5;
    load_next();
    cur = joined();
    load_next();
    pos = 0;
    buf = 0;
    nb = 0;
    taken = 0;
    refill();
    drop = (uint32_t)(bit & 31);
    buf <<= drop;
    nb -= (int)drop;
  }
  // bits consumed since the start
  __device__ __forceinline__ uint64_t used() const { return 32ull * taken - (uint64_t)nb - drop; }
  __device__ __forceinline__ void refill() {
    if (nb <= 32) {
      const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)cur, (int)pos);
      buf |= (uint64_t)w << (32 - nb);
      nb += 32;
      taken++;
      if (++pos == BZG_WAVE) {
        cur = joined();
        load_next();
        pos = 0;
      }
    }
  }
  __device__ __forceinline__ uint32_t peek(int k) const { return (uint32_t)(buf >> (64 - k)); }
  __device__ __forceinline__ void skip(int k) {
    buf <<= k;
    nb -= k;
  }
  __device__ __forceinline__ uint32_t get(int k) {  // k <= 24
    refill();
    const uint32_t v = peek(k);
    skip(k);
    return v;
  }
};

constexpr uint32_t MAX_SEL = 18002;  // selectors kept per block (more are read and dropped)
constexpr int DEC_MAXLEN = 20;
constexpr uint32_t OBUF = 4096;    // output bytes staged per inverse-MTF chunk
constexpr uint32_t MTF_CH = 4096;  // symbols per inverse-MTF chunk

// Huffman decoding a step at a time: a step decodes up to one group's
// remaining codes inside a span of SPAN bits.  Lane l evaluates bit
// positions PSTEP*l .. PSTEP*l + PSTEP-1 of the span as if a code started
// there.  The map position -> next code start is composed with itself
// (pointer doubling), and lane l follows it l times from the step's start.
// A map entry holds 4 * the target position (high half) and the symbol of
// the code it passed last (low half), which composition carries along: lane
// l ends with code l's start and code l-1's symbol.
constexpr uint32_t PSTEP = 8;
constexpr uint32_t SPAN = PSTEP * BZG_WAVE;        // 512 bit positions
constexpr uint32_t JSENT = SPAN + DEC_MAXLEN;      // beyond the span (a fixed point of the map)
constexpr uint32_t JTAB = JSENT + 4;               // map entries, a multiple of 8
constexpr uint32_t LUT_BAD = 0x8000u | (1u << 9) | 511u;  // no code here: length 1, symbol 0x81FF
constexpr uint32_t SYM_BAD = LUT_BAD & 0x81FFu;
constexpr uint32_t SYM_BEYOND = 0x7FFFu;           // the code passed started past the span
constexpr uint32_t NLONG = DEC_MAXLEN - DEC_LUT_BITS;     // code lengths past the first-level table

// Until a block's last-to-first map is built, its range of the map (4 bytes
// per row of its capacity) holds its symbols (uint16, from the start) and
// their starting-list indices (bytes, from 2 * cap on): each block's scratch
// stays inside its own range.
__device__ __forceinline__ uint16_t* blk_syms(uint32_t* FL, const DecBlk& B) { return (uint16_t*)(FL + B.l_off); }
__device__ __forceinline__ uint8_t* blk_q(uint32_t* FL, const DecBlk& B) {
  return (uint8_t*)(FL + B.l_off) + 2 * (size_t)B.cap;
}

// One wave per block: header, symbol map, selectors, code tables, then
// every Huffman code up to end-of-block, a group per step (first-level
// table, then the canonical limits for longer codes).  Writes the block's symbols (RUNA/RUNB digits and
// move-to-front positions + 1, uint16, at the start of the block's map range),
// their count, the move-to-front list it starts from (the in-use bytes,
// ascending), origPtr and the stored CRC.  The move-to-front and run
// decoding run afterwards, in parallel over chunks.
__global__ __launch_bounds__(BZG_WAVE) void k_dec_block(const uint8_t* __restrict__ in, uint64_t n_in,
                                                        const DecBlk* __restrict__ blks,
                                                        const uint32_t* __restrict__ order,
                                                        uint32_t* __restrict__ FL, uint32_t* __restrict__ n_syms,
                                                        uint8_t* __restrict__ mtf0,
                                                        uint32_t* __restrict__ out_orig,
                                                        uint32_t* __restrict__ out_crc, uint32_t* __restrict__ err) {
  __shared__ uint16_t lut[MAXG][1u << DEC_LUT_BITS];
  __shared__ uint16_t perm[MAXG][MAXA];
  __shared__ __align__(4) uint8_t unseq[256];
  __shared__ int32_t lim20[MAXG][32];            // left-aligned limits, per length
  __shared__ int32_t sbase[MAXG][DEC_MAXLEN + 2];  // start - first code, per length
  // what only the table building uses shares its LDS with what only the
  // symbol steps use (fewer bytes per workgroup, more workgroups per CU)
  __shared__ union {
    struct {
      int32_t limit[MAXG][DEC_MAXLEN + 2];
      uint32_t first[MAXG][DEC_MAXLEN + 2], start[MAXG][DEC_MAXLEN + 2];
      uint8_t lens[MAXG][MAXA];
      uint32_t srun[DEC_MAXLEN + 2];
    } build;
    struct {
      uint32_t ring[2 * BZG_WAVE];                 // two 64-dword windows of the stream
      __align__(16) uint32_t jt[2][JTAB];          // next-code-start maps (ping-pong)
    } step;
  } ls;
  auto& limit = ls.build.limit;
  auto& first = ls.build.first;
  auto& start = ls.build.start;
  auto& lens = ls.build.lens;
  auto& srun = ls.build.srun;
  auto& ring = ls.step.ring;
  auto& jt = ls.step.jt;
  const uint32_t b = order[blockIdx.x];  // the longest blocks first
  const DecBlk B = blks[b];
  uint16_t* Sb = blk_syms(FL, B);
  const uint32_t ln = lane();
  BitIn r{in, n_in};
  r.start(B.start);
  uint32_t bad = 0;
  const uint32_t crc_hi = r.get(16);
  const uint32_t crc = (crc_hi << 16) | r.get(16);
  const uint32_t rnd = r.get(1);
  const uint32_t orig = r.get(24);
  bad |= rnd;  // randomised blocks (an obsolete encoder option) are not decoded
  // symbol map
  const uint32_t r16 = r.get(16);
  uint32_t nin = 0;
  for (int i = 0; i < 16; i++) {
    if (!((r16 >> (15 - i)) & 1u)) continue;
    const uint32_t bits = r.get(16);
    for (int j = 0; j < 16; j++)
      if ((bits >> (15 - j)) & 1u) {
        if (ln == 0) unseq[nin] = (uint8_t)(16 * i + j);
        nin++;
      }
  }
  bad |= nin == 0;
  const int a = (int)nin + 2;
  const int G = (int)r.get(3);
  const uint32_t nsel = r.get(15);
  bad |= (G < 2) | (G > MAXG) | (nsel == 0);
  // selectors: checked here and decoded again, one per group, in the symbol
  // loop by a second reader (unary table positions, move-to-front over the
  // tables)
  const uint64_t sel_bit = B.start + r.used();
  for (uint32_t s = 0; s < nsel && !bad; s++) {
    uint32_t j = 0;
    while (r.get(1)) {
      j++;
      if (j >= (uint32_t)G) {
        bad = 1;
        break;
      }
    }
  }
  const uint32_t nsel_kept = min(nsel, MAX_SEL);
  // code lengths, delta coded
  for (int t = 0; t < G && !bad; t++) {
    int cur = (int)r.get(5);
    for (int i = 0; i < a; i++) {
      for (;;) {
        if (cur < 1 || cur > DEC_MAXLEN) {
          bad = 1;
          break;
        }
        if (!r.get(1)) break;
        cur += r.get(1) ? -1 : 1;
      }
      if (bad) break;
      if (ln == 0) lens[t][i] = (uint8_t)cur;
    }
  }
  __syncthreads();
  // the list the block's move-to-front decoding starts from
  for (uint32_t i = nin + ln; i < 256u; i += BZG_WAVE) unseq[i] = 0;
  __syncthreads();
  ((uint32_t*)(mtf0 + (size_t)b * 256))[ln] = ((const uint32_t*)unseq)[ln];
  // decoding tables: canonical first codes, limits, symbols by length
  if (!bad) {
    for (int t = 0; t < G; t++) {
      if (ln < DEC_MAXLEN + 2) srun[ln] = 0;
      __syncthreads();
      for (int i = ln; i < a; i += BZG_WAVE) atomicAdd(&srun[lens[t][i]], 1u);
      __syncthreads();
      if (ln == 0) {
        uint32_t code = 0, st = 0;
        for (int l = 1; l <= DEC_MAXLEN; l++) {
          const uint32_t c = srun[l];
          first[t][l] = code;
          start[t][l] = st;
          limit[t][l] = (int32_t)(code + c) - 1;
          // a 20-bit prefix v holds a code of length <= l iff v <= lim20[l];
          // these rise with l (any counts), so the length is found by counting
          lim20[t][l] = (int32_t)((code + c) << (DEC_MAXLEN - l)) - 1;
          sbase[t][l] = (int32_t)st - (int32_t)code;
          code = (code + c) << 1;
          st += c;
        }
      }
      __syncthreads();
      if (ln < DEC_MAXLEN + 2) srun[ln] = 0;
      __syncthreads();
      // symbols of each length in symbol order: ranks by ballots, 64 at a time
      for (int k = 0; k * BZG_WAVE < a; k++) {
        const int v = k * BZG_WAVE + (int)ln;
        const bool ok = v < a;
        const uint32_t l = ok ? lens[t][v] : 0u;
        const uint64_t peers = match_digit8(l, __ballot(ok));
        const uint32_t before = srun[l];
        if (ok) perm[t][start[t][l] + before + (uint32_t)__popcll(peers & lanemask_lt())] = (uint16_t)v;
        if (ok && (uint32_t)(__ffsll((long long)peers) - 1) == ln) srun[l] = before + (uint32_t)__popcll(peers);
        __syncthreads();
      }
      // first-level table: the shortest code length whose limit admits the prefix
      for (uint32_t x = ln; x < (1u << DEC_LUT_BITS); x += BZG_WAVE) {
        uint16_t e = 0;
        for (int l = 1; l <= (int)DEC_LUT_BITS; l++) {
          const int32_t v = (int32_t)(x >> (DEC_LUT_BITS - l));
          if (v <= limit[t][l]) {
            const uint32_t idx = start[t][l] + (uint32_t)v - first[t][l];
            e = (uint16_t)(idx < (uint32_t)a ? (perm[t][idx] | (l << 9)) : LUT_BAD);
            break;
          }
        }
        lut[t][x] = e;
      }
    }
  }
  __syncthreads();
  // symbols.  Each group of GROUP codes uses the table its selector names;
  // a step decodes the group's remaining codes that start inside the next
  // SPAN bits (all of them unless the codes average over SPAN/GROUP bits).
  // Lane k+1 of a step holds its k-th code; the step's symbols are stored
  // together (coalesced).  A block has at most as many symbols as bytes.
  // The workgroup is one wave, whose LDS accesses take effect in program
  // order: the step's phases need compiler fences only.
  const uint32_t cap = B.cap;
  uint32_t cnt = 0, gsel = 0, rem = 0, t = 0;
  const uint32_t eob = (uint32_t)a - 1;
  uint64_t bit = B.start + r.used();  // the first code
  BitIn rs{in, n_in};
  rs.start(sel_bit);
  uint32_t lst = 0x543210u;  // table list, 4 bits per entry, front in the low bits
  bool ended = false;
  int32_t lv = 0;  // lane l: left-aligned limit of length l of the group's table
  for (uint32_t i = SPAN + ln; i < JTAB; i += BZG_WAVE) {
    jt[0][i] = (4 * JSENT << 16) | SYM_BEYOND;
    jt[1][i] = (4 * JSENT << 16) | SYM_BEYOND;
  }
  // the stream as 64-dword windows: ring slot (w & 1) holds window w; the
  // ring holds the windows of `bit` and the next, pb the one after
  uint32_t wr = (uint32_t)(bit >> 11);
  uint32_t pb[4];
  auto win_load = [&](uint64_t w) {
    const uint64_t q = 4 * (BZG_WAVE * w + ln);
#pragma unroll
    for (int i = 0; i < 4; i++) pb[i] = in[min(q + i, n_in - 1)];
  };
  auto win_put = [&](uint64_t w) {
    ring[BZG_WAVE * (uint32_t)(w & 1) + ln] = (pb[0] << 24) | (pb[1] << 16) | (pb[2] << 8) | pb[3];
  };
  auto put_row = [&](uint32_t* row, const uint32_t (&v)[PSTEP]) {
    ((uint4*)row)[0] = make_uint4(v[0], v[1], v[2], v[3]);
    ((uint4*)row)[1] = make_uint4(v[4], v[5], v[6], v[7]);
  };
  auto lds_order = [] {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  win_load(wr);
  win_put(wr);
  win_load(wr + 1ull);
  win_put(wr + 1ull);
  win_load(wr + 2ull);
  bad = uni(bad);
  __syncthreads();
  while (!bad && !ended) {
    if (rem == 0) {
      if (gsel >= nsel_kept) {
        bad = 1;
        break;
      }
      // j ones and a zero (j < G, checked above): table at list position j
      rs.refill();
      const uint32_t j = (uint32_t)__builtin_clz(~rs.peek(32) | 1u);
      rs.skip((int)j + 1);
      t = (lst >> (4 * j)) & 15u;
      const uint32_t below = lst & ((1u << (4 * j)) - 1u);
      lst = (lst & ~((1u << (4 * j + 4)) - 1u)) | (below << 4) | t;
      gsel++;
      rem = GROUP;
      lv = lim20[t][ln & 31u];
    }
    // this lane's 32 bits from span position PSTEP*ln
    const uint64_t q = bit + PSTEP * ln;
    const uint32_t dq = (uint32_t)(q >> 5);
    const uint64_t hl = ((uint64_t)ring[dq & (2 * BZG_WAVE - 1)] << 32) | ring[(dq + 1) & (2 * BZG_WAVE - 1)];
    const uint32_t w = (uint32_t)(hl >> (32 - ((uint32_t)q & 31u)));
    uint32_t jv[PSTEP];
#pragma unroll
    for (uint32_t i = 0; i < PSTEP; i++) jv[i] = lut[t][(w >> (32 - DEC_LUT_BITS - i)) & ((1u << DEC_LUT_BITS) - 1u)];
    uint32_t slow = 0;
#pragma unroll
    for (uint32_t i = 0; i < PSTEP; i++) {
      slow |= (jv[i] == 0 ? 1u : 0u) << i;
      jv[i] = ((4 * (PSTEP * ln + i + ((jv[i] >> 9) & 31u))) << 16) | (jv[i] & 0x81FFu);
    }
    uint32_t* jrow = &jt[0][PSTEP * ln];
    put_row(jrow, jv);
    if (__ballot(slow != 0)) {
      // codes longer than the first-level table: the first length whose
      // limit admits the 20-bit prefix; the entries are rewritten in place
      int32_t lim[DEC_MAXLEN - DEC_LUT_BITS];
#pragma unroll
      for (uint32_t l = 0; l < DEC_MAXLEN - DEC_LUT_BITS; l++)
        lim[l] = __builtin_amdgcn_readlane(lv, (int)(DEC_LUT_BITS + 1 + l));
      while (slow) {
        const uint32_t i = (uint32_t)__builtin_ctz(slow);
        slow &= slow - 1u;
        const uint32_t v = (w >> (32 - DEC_MAXLEN - i)) & ((1u << DEC_MAXLEN) - 1u);
        uint32_t zn = DEC_LUT_BITS + 1;
#pragma unroll
        for (uint32_t l = 0; l + 1 < DEC_MAXLEN - DEC_LUT_BITS; l++) zn += (int32_t)v > lim[l] ? 1u : 0u;
        const uint32_t idx = (uint32_t)(sbase[t][zn] + (int32_t)(v >> (DEC_MAXLEN - zn)));
        const uint32_t ee = (int32_t)v <= lim[DEC_MAXLEN - DEC_LUT_BITS - 1] && idx < (uint32_t)a
                                ? (perm[t][idx] | (zn << 9))
                                : LUT_BAD;
        jrow[i] = ((4 * (PSTEP * ln + i + ((ee >> 9) & 31u))) << 16) | (ee & 0x81FFu);
      }
      const uint4 r0 = ((const uint4*)jrow)[0], r1 = ((const uint4*)jrow)[1];
      jv[0] = r0.x;
      jv[1] = r0.y;
      jv[2] = r0.z;
      jv[3] = r0.w;
      jv[4] = r1.x;
      jv[5] = r1.y;
      jv[6] = r1.z;
      jv[7] = r1.w;
    }
    lds_order();
    // doubling: table k maps a position to the start 2^k codes on; lane ln
    // takes table k when bit k of ln is set
    uint32_t x = 0;  // 4 * code ln's start (high half), code ln-1's symbol
#pragma unroll
    for (uint32_t k = 0; k < 6; k++) {
      const char* A = (const char*)jt[k & 1];
      const uint32_t xa = *(const uint32_t*)(A + (x >> 16));
      if (k < 5) {
#pragma unroll
        for (uint32_t i = 0; i < PSTEP; i++) jv[i] = *(const uint32_t*)(A + (jv[i] >> 16));
      }
      x = (ln >> k) & 1u ? xa : x;
      if (k < 5) {
        put_row(&jt[(k + 1) & 1][PSTEP * ln], jv);
        lds_order();
      }
    }
    // codes that start inside the span are exact (the map saturates past it)
    const uint32_t sym = x & 0xFFFFu, xs = x >> 18;
    const bool ok = ln >= 1 && ln <= rem && sym != SYM_BEYOND;
    const uint64_t vm = __ballot(ok);
    const uint64_t em = __ballot(ok && sym == eob);
    const uint64_t im = __ballot(ok && sym == SYM_BAD);
    uint32_t m = (uint32_t)__popcll(vm);  // lanes 1 .. m
    uint32_t nl = m;                      // the lane holding the next start
    if (em) {
      nl = (uint32_t)__builtin_ctzll(em);
      m = nl - 1;
      ended = true;
    }
    const uint32_t nx = (uint32_t)__builtin_amdgcn_readlane((int)xs, (int)nl);
    if ((im & ((2ull << m) - 2ull)) | (cnt + m > cap)) {
      bad = 1;
      break;
    }
    // (symbols are < a: a literal's list position, sym - 1, is < nin)
    if (ln >= 1 && ln <= m) Sb[cnt + ln - 1] = (uint16_t)sym;
    cnt += m;
    rem -= m;
    bit += nx;
    if ((uint32_t)(bit >> 11) != wr) {  // at most one window per step
      wr++;
      win_put(wr + 1ull);
      win_load(wr + 2ull);
    }
    lds_order();
  }
  // the block's bits must end exactly where the next marker starts
  bad |= !ended | (cnt == 0);  // a block holds at least one byte
  bad |= (bit != B.end);
  if (ln == 0) {
    n_syms[b] = bad ? 0u : cnt;
    out_orig[b] = orig;
    out_crc[b] = crc;
    if (bad) atomicOr(err, ERR_STREAM);
  }
}

// ------------------------------------------- move-to-front, run decoding

// List entry i (i < 256) of a move-to-front list held four entries per lane
// (entry 4*lane + k in byte k), moved to the front; returns it.
__device__ __forceinline__ uint32_t mtf_take(uint32_t& stk, uint32_t i) {
  const uint32_t ln = lane();
  const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int)stk, (int)(i >> 2));
  const uint32_t uc = (word >> (8 * (i & 3u))) & 255u;
  // positions 0 .. i-1 move up one, uc goes to the front
  const uint32_t prev = wave_shr1(0u, stk);
  const uint32_t up = (stk << 8) | (prev >> 24);
  const int take = min(max((int)i - 4 * (int)ln + 1, 0), 4);  // bytes of this lane at positions <= i
  const uint32_t m = take == 4 ? 0xFFFFFFFFu : ((1u << (8 * take)) - 1u);
  stk = (up & m) | (stk & ~m);
  if (ln == 0) stk = (stk & ~255u) | uc;
  return uc;
}

// The first symbol at or after s that starts an item (a literal, or the
// first digit of a run): s itself unless s continues a run begun before it.
// Runs are at most a few dozen digits; a longer one is flagged.
__device__ __forceinline__ uint32_t item_start(const uint16_t* __restrict__ S, uint32_t n, uint32_t s,
                                               uint32_t* __restrict__ err) {
  if (s == 0 || s >= n) return min(s, n);
  // window lane w: symbol s - 1 + w (past the end: taken as a literal)
  const uint32_t i = s - 1 + lane();
  const uint64_t lit = __ballot(i >= n || S[i] >= 2u);
  // symbol s + k starts an item when it, or the one before it, is a literal
  const uint64_t st = (lit | (lit >> 1)) & ~(1ull << 63);
  if (!st) {
    if (lane() == 0) atomicOr(err, ERR_STREAM);
    return n;
  }
  return min(s + (uint32_t)(__ffsll((long long)st) - 1), n);
}

// Chunk slot j of the per-block chunk layout: its block and index there.
struct MtfChunk {
  uint32_t b, c;
};
__device__ __forceinline__ MtfChunk mtf_chunk(const uint64_t* __restrict__ ch0, uint32_t nb, uint64_t j,
                                              const uint32_t* __restrict__ bl) {
  MtfChunk k;
  uint32_t lo = 0, hi = nb;  // ch0[lo] <= j < ch0[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (ch0[mid] <= j) lo = mid;
    else hi = mid;
  }
  k.b = bl[lo];
  k.c = (uint32_t)(j - ch0[lo]);
  return k;
}

__device__ void mtf_perm_chunk(uint64_t j, const DecBlk* __restrict__ blks, const uint64_t* __restrict__ ch0,
                               uint32_t nb, const uint32_t* __restrict__ bl, uint32_t* __restrict__ FL,
                               const uint32_t* __restrict__ n_syms,
                               uint8_t* __restrict__ T,
                               uint32_t* __restrict__ cs, uint32_t* __restrict__ ce, uint32_t* __restrict__ clen,
                               uint32_t* __restrict__ err) {
  const MtfChunk k = mtf_chunk(ch0, nb, j, bl);
  const uint32_t n = n_syms[k.b];
  if ((uint64_t)k.c * MTF_CH >= n) return;
  const DecBlk B = blks[k.b];
  const uint16_t* S = blk_syms(FL, B);
  const uint32_t ln = lane();
  const uint32_t s = item_start(S, n, k.c * MTF_CH, err);
  const uint32_t e = item_start(S, n, (uint32_t)min((uint64_t)(k.c + 1) * MTF_CH, (uint64_t)n), err);
  uint8_t* Qb = blk_q(FL, B);
  uint32_t stk = (4u * ln) | ((4u * ln + 1u) << 8) | ((4u * ln + 2u) << 16) | ((4u * ln + 3u) << 24);
  uint64_t out = 0, run = 0;
  uint32_t rk = 0;
  for (uint32_t base = s; base < e; base += BZG_WAVE) {
    const uint32_t m = min((uint32_t)BZG_WAVE, e - base);
    const uint32_t v = ln < m ? S[base + ln] : 0u;
    uint32_t qv = 0;  // lane q: the starting-list index of symbol base + q's byte
    for (uint32_t q = 0; q < m; q++) {
      const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)q);
      uint32_t from;
      if (x <= 1u) {  // RUNA / RUNB: a digit of the zero run, least significant first
        run += (uint64_t)(x + 1u) << min(rk, 40u);
        rk++;
        from = (uint32_t)__builtin_amdgcn_readlane((int)stk, 0) & 255u;  // the run repeats the front
      } else {
        out += run + 1u;
        run = 0;
        rk = 0;
        from = mtf_take(stk, x - 1u);
      }
      qv = ln == q ? from : qv;
    }
    if (ln < m) Qb[base + ln] = (uint8_t)qv;
  }
  out += run;
  const bool bad = rk > 40u || out > B.cap;
  ((uint32_t*)(T + B.l_off + (size_t)k.c * 256))[ln] = stk;
  if (ln == 0) {
    cs[j] = s;
    ce[j] = e;
    clen[j] = bad ? B.cap + 1u : (uint32_t)out;
  }
}

// A block's chunk c holds the items that start among its symbols
// [c*MTF_CH, (c+1)*MTF_CH).  Move-to-front decoding of a chunk moves list
// positions the same way whatever the list holds, so each chunk's effect is
// a permutation of positions, found here by decoding it on the identity
// list (one wave per chunk); chunks are then chained by composing them.
// Also the chunk's item range and output length, and for every symbol the
// index in the chunk's starting list of the byte it stands for (the front,
// for a run digit), so that the bytes follow from that list without
// decoding again.  Per block, the
// permutations sit in the first cap/MTF_CH + 1 256-byte slots of its T range
// and the chunks' starting lists in the next as many.
__global__ __launch_bounds__(BZG_WAVE) void k_dec_mtf_perm(const DecBlk* __restrict__ blks,
                                                           const uint64_t* __restrict__ ch0, uint32_t nb,
                                                           const uint32_t* __restrict__ bl, uint32_t* __restrict__ FL,
                                                           const uint32_t* __restrict__ n_syms,
                                                           uint8_t* __restrict__ T, uint32_t* __restrict__ cs,
                                                           uint32_t* __restrict__ ce, uint32_t* __restrict__ clen,
                                                           uint32_t* __restrict__ err) {
  const uint64_t total = ch0[nb];
  for (uint64_t j = blockIdx.x; j < total; j += gridDim.x)
    mtf_perm_chunk(j, blks, ch0, nb, bl, FL, n_syms, T, cs, ce, clen, err);
}
// Per block (one wave): each chunk's starting list and output offset, by
// composing the chunk permutations in order from the block's first list;
// then the block's length and its checks (at least one byte, origPtr inside).
__global__ __launch_bounds__(BZG_WAVE) void k_dec_mtf_scan(const DecBlk* __restrict__ blks,
                                                           const uint64_t* __restrict__ ch0,
                                                           const uint32_t* __restrict__ bl,
                                                           const uint32_t* __restrict__ n_syms,
                                                           const uint8_t* __restrict__ mtf0, uint8_t* __restrict__ T,
                                                           const uint32_t* __restrict__ clen,
                                                           uint32_t* __restrict__ coff,
                                                           const uint32_t* __restrict__ orig,
                                                           uint32_t* __restrict__ n_rows, uint32_t* __restrict__ err) {
  __shared__ __align__(4) uint8_t lst[256];
  const uint32_t bi = blockIdx.x, b = bl[bi], ln = lane();
  const DecBlk B = blks[b];
  const uint32_t n = n_syms[b];
  const uint32_t nch = (n + MTF_CH - 1) / MTF_CH, slots = B.cap / MTF_CH + 1;
  const uint64_t j0 = ch0[bi];
  uint8_t* Tb = T + B.l_off;
  ((uint32_t*)lst)[ln] = ((const uint32_t*)(mtf0 + (size_t)b * 256))[ln];
  __syncthreads();
  uint64_t acc = 0;
  for (uint32_t c0 = 0; c0 < nch; c0 += BZG_WAVE) {
    // output offsets of 64 chunks at once
    const uint32_t c = c0 + ln;
    const uint64_t len = c < nch ? clen[j0 + c] : 0u;
    const uint64_t inc = wave_incl_sum(len);
    if (c < nch) coff[j0 + c] = (uint32_t)min(acc + inc - len, (uint64_t)B.cap + 1u);
    acc += wave_last(inc);
    const uint32_t m = min((uint32_t)BZG_WAVE, nch - c0);
    uint32_t pw = ((const uint32_t*)(Tb + (size_t)c0 * 256))[ln];
    for (uint32_t q = 0; q < m; q++) {
      const uint32_t cc = c0 + q;
      // this chunk's permutation in hand, the next one's loaded
      const uint32_t pn = q + 1 < m ? ((const uint32_t*)(Tb + (size_t)(cc + 1) * 256))[ln] : 0u;
      const uint32_t cur = ((const uint32_t*)lst)[ln];
      ((uint32_t*)(Tb + (size_t)(slots + cc) * 256))[ln] = cur;
      const uint32_t nw = (uint32_t)lst[pw & 255u] | ((uint32_t)lst[(pw >> 8) & 255u] << 8) |
                          ((uint32_t)lst[(pw >> 16) & 255u] << 16) | ((uint32_t)lst[pw >> 24] << 24);
      __syncthreads();
      ((uint32_t*)lst)[ln] = nw;
      __syncthreads();
      pw = pn;
    }
  }
  const bool bad = n != 0 && (acc == 0 || acc > B.cap || orig[b] >= acc);
  if (ln == 0) {
    n_rows[b] = n == 0 || bad ? 0u : (uint32_t)acc;
    if (bad) atomicOr(err, ERR_STREAM);
  }
}

// One wave per chunk, 64 symbols a step: every symbol's byte is its
// starting-list entry, so a step finds each run's length (a segmented sum of
// its digits' weights, a run carried across steps), each item's output
// offset (a scan of the counts), and writes the bytes (literals one per
// lane, runs by their last digit's lane, long runs by the whole wave).
__device__ void mtf_emit_chunk(uint64_t j, const DecBlk* __restrict__ blks, const uint64_t* __restrict__ ch0,
                               uint32_t nb, const uint32_t* __restrict__ bl, uint32_t* __restrict__ FL,
                               const uint32_t* __restrict__ n_syms,
                               const uint8_t* __restrict__ T,
                               const uint32_t* __restrict__ cs, const uint32_t* __restrict__ ce,
                               const uint32_t* __restrict__ coff, const uint32_t* __restrict__ n_rows,
                               uint8_t* __restrict__ L, uint8_t* lst) {
  const MtfChunk k = mtf_chunk(ch0, nb, j, bl);
  const uint32_t n = n_syms[k.b], rows = n_rows[k.b];
  if ((uint64_t)k.c * MTF_CH >= n || rows == 0) return;  // past the symbols, or a bad block
  const DecBlk B = blks[k.b];
  const uint16_t* S = blk_syms(FL, B);
  const uint8_t* Qb = blk_q(FL, B);
  const uint32_t ln = lane(), slots = B.cap / MTF_CH + 1;
  ((uint32_t*)lst)[ln] = ((const uint32_t*)(T + B.l_off + (size_t)(slots + k.c) * 256))[ln];
  __syncthreads();
  const uint32_t s = cs[j], e = ce[j];
  uint8_t* out = L + B.l_off + coff[j];  // the block's length checks bound every chunk inside it
  uint64_t acc = 0;  // bytes written
  // a run going on from the step before: its digits so far and their sum
  uint32_t ck = 0;
  uint64_t cv = 0;
  bool cdig = false;
  for (uint32_t base = s; base < e; base += BZG_WAVE) {
    const uint32_t m = min((uint32_t)BZG_WAVE, e - base);
    const bool valid = ln < m;
    const uint32_t x = valid ? S[base + ln] : 2u;
    const uint32_t q = valid ? Qb[base + ln] : 0u;
    const uint32_t xn = base + BZG_WAVE < e ? S[base + BZG_WAVE] : 2u;  // the symbol after the step
    const bool dig = valid && x <= 1u;
    const uint64_t digm = __ballot(dig);
    const bool prevdig = ln == 0 ? cdig : ((digm >> (ln - 1)) & 1ull) != 0;
    const uint64_t startm = __ballot(dig && !prevdig);
    const uint64_t le = startm & (ln == BZG_WAVE - 1 ? ~0ull : ((2ull << ln) - 1ull));
    const int ls = le ? 63 - (int)__clzll((long long)le) : -1;  // the run's first digit in this step
    const uint32_t kk = ls >= 0 ? ln - (uint32_t)ls : ln + ck;   // the digit's place in its run
    const uint64_t v = dig ? (uint64_t)(x + 1u) << min(kk, 40u) : 0ull;
    const uint64_t inc = wave_incl_sum(v);
    const int src = ls > 0 ? ls - 1 : 0;
    const uint64_t at = (uint64_t)(uint32_t)__shfl((int)(uint32_t)inc, src) |
                        ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(inc >> 32), src) << 32);
    const uint64_t part = ls > 0 ? inc - at : ls == 0 ? inc : inc + cv;  // the run's sum up to this digit
    const bool nextdig = ln == BZG_WAVE - 1 ? xn <= 1u : ((digm >> (ln + 1)) & 1ull) != 0;
    const bool run_end = dig && !nextdig;
    const uint64_t cnt = !valid ? 0ull : dig ? (run_end ? part : 0ull) : 1ull;
    // a run going on into the next step
    const bool last_dig = ((digm >> (BZG_WAVE - 1)) & 1ull) != 0 && xn <= 1u;
    const uint32_t ck_n = (uint32_t)__builtin_amdgcn_readlane((int)kk, BZG_WAVE - 1) + 1u;
    const uint64_t cv_n = wave_last(part);
    cdig = last_dig;
    ck = last_dig ? ck_n : 0u;
    cv = last_dig ? cv_n : 0ull;
    const uint64_t ci = wave_incl_sum(cnt);
    const uint64_t o = acc + ci - cnt;
    acc += wave_last(ci);
    const uint8_t by = lst[q];
    if (valid && !dig) out[o] = by;
    if (run_end && part <= BZG_WAVE)
      for (uint32_t i = 0; i < (uint32_t)part; i++) out[o + i] = by;
    uint64_t bigm = __ballot(run_end && part > BZG_WAVE);
    while (bigm) {  // long runs: the whole wave writes each
      const int l = (int)(__ffsll((long long)bigm) - 1);
      bigm &= bigm - 1;
      const uint64_t R = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)part, l) |
                         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(part >> 32), l) << 32);
      const uint64_t oo = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)o, l) |
                          ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(o >> 32), l) << 32);
      const uint8_t b8 = (uint8_t)__builtin_amdgcn_readlane((int)by, l);
      for (uint64_t i = ln; i < R; i += BZG_WAVE) out[oo + i] = b8;
    }
  }
}

__global__ __launch_bounds__(BZG_WAVE) void k_dec_mtf_emit(const DecBlk* __restrict__ blks,
                                                           const uint64_t* __restrict__ ch0, uint32_t nb,
                                                           const uint32_t* __restrict__ bl, uint32_t* __restrict__ FL,
                                                           const uint32_t* __restrict__ n_syms,
                                                           const uint8_t* __restrict__ T,
                                                           const uint32_t* __restrict__ cs,
                                                           const uint32_t* __restrict__ ce,
                                                           const uint32_t* __restrict__ coff,
                                                           const uint32_t* __restrict__ n_rows,
                                                           uint8_t* __restrict__ L) {
  __shared__ __align__(4) uint8_t lst[256];
  const uint64_t total = ch0[nb];
  for (uint64_t j = blockIdx.x; j < total; j += gridDim.x) {
    mtf_emit_chunk(j, blks, ch0, nb, bl, FL, n_syms, T, cs, ce, coff, n_rows, L, lst);
    __syncthreads();
  }
}

// ------------------------------------------------------ inverse BWT map

// The block owning flat slot j of a per-block slot layout (offsets s0[0..nb]).
__device__ __forceinline__ uint32_t owner_of(const uint64_t* __restrict__ s0, uint32_t nb, uint64_t j) {
  uint32_t lo = 0, hi = nb;  // s0[lo] <= j < s0[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (s0[mid] <= j) lo = mid;
    else hi = mid;
  }
  return lo;
}
// The same for a workgroup of consecutive slots: one search for its first
// slot (workgroup-uniform), then each thread steps over the few blocks its
// slot lies past.
__device__ __forceinline__ uint32_t owner_of_wg(const uint64_t* __restrict__ s0, uint32_t nb, uint64_t j) {
  uint32_t b = owner_of(s0, nb, j - threadIdx.x);
  while (b + 1 < nb && s0[b + 1] <= j) b++;
  return b;
}

// FL of one block: the row that holds, in the last column, the k-th
// occurrence of the byte that is first in row C[byte] + k -- a stable
// counting sort of the column.  Each entry carries that byte in its top 8
// bits (rows < 2^24), so the walks read one array.  The column is cut into
// chunks of FL_CH rows (a workgroup each; slots planned from the block's
// capacity, those past its length idle): byte counts per chunk, then per
// block their offsets, then every chunk writes its rows, each wave its own
// FL_SUB rows 64 at a time.
constexpr uint32_t FL_CH = 65536;
constexpr uint32_t FL_NW = NT / BZG_WAVE;
constexpr uint32_t FL_SUB = FL_CH / FL_NW;
constexpr uint32_t FL_BATCH = 16 * BZG_WAVE;  // column bytes a wave stages at a time

// The block of every FL chunk (a thread per block): the chunk kernels are
// persistent over the chunks that exist.
__global__ void k_dec_fl_owner(const uint64_t* __restrict__ off, uint32_t nb, uint32_t* __restrict__ owner) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  for (uint64_t j = off[b]; j < off[b + 1]; j++) owner[j] = b;
}

// Byte counts of rows [lo, hi) of a block's column into h (LDS atomics, 16
// bytes per thread a step; block ranges are 16-byte aligned and padded).
__device__ __forceinline__ void fl_count(const uint8_t* __restrict__ Lb, uint32_t lo, uint32_t hi, uint32_t t,
                                         uint32_t nt, uint32_t* h) {
  for (uint32_t k = lo + 16 * t; k < hi; k += 16 * nt) {
    const uint4 v = *(const uint4*)(Lb + k);
    const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (uint32_t q = 0; q < 16; q++)
      if (k + q < hi) atomicAdd(&h[(wv[q / 4] >> (8 * (q % 4))) & 255u], 1u);
  }
}

__global__ __launch_bounds__(NT) void k_dec_fl_count(const DecBlk* __restrict__ blks, uint32_t nb,
                                                     const uint32_t* __restrict__ bl, const uint64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ owner, const uint8_t* __restrict__ L,
                                                     const uint32_t* __restrict__ n_rows, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[FL_NW][256];
  const uint32_t tid = threadIdx.x, w = tid / BZG_WAVE;
  const uint64_t total = off[nb];
  for (uint64_t j = blockIdx.x; j < total; j += gridDim.x) {
    const uint32_t bi = owner[j], b = bl[bi], c = (uint32_t)(j - off[bi]), n = n_rows[b];
    for (uint32_t q = 0; q < FL_NW; q++) h[q][tid] = 0;
    __syncthreads();
    const uint32_t lo = c * FL_CH, hi = min(n, lo + FL_CH);
    fl_count(L + blks[b].l_off, lo, hi, tid, NT, h[w]);
    __syncthreads();
    uint32_t t = 0;
    for (uint32_t q = 0; q < FL_NW; q++) t += h[q][tid];
    cnt[j * 256 + tid] = t;
    __syncthreads();
  }
}

// Per block (a workgroup, a thread per byte): each chunk's first row per
// byte -- the byte's start in the first column plus the chunks before.
__global__ __launch_bounds__(NT) void k_dec_fl_scan(const uint64_t* __restrict__ off, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  const uint32_t b = blockIdx.x, d = threadIdx.x;
  const uint32_t nch = (uint32_t)(off[b + 1] - off[b]);
  uint32_t* cb = cnt + off[b] * 256;
  uint32_t acc = 0;
  for (uint32_t c = 0; c < nch; c++) {
    const uint32_t v = cb[c * 256 + d];
    cb[c * 256 + d] = acc;
    acc += v;
  }
  uint32_t tot;
  const uint32_t C = block_excl_sum<uint32_t, NT>(acc, sh, &tot);
  for (uint32_t c = 0; c < nch; c++) cb[c * 256 + d] += C;
}

__global__ __launch_bounds__(NT) void k_dec_fl(const DecBlk* __restrict__ blks, uint32_t nb,
                                               const uint32_t* __restrict__ bl, const uint64_t* __restrict__ off,
                                               const uint32_t* __restrict__ owner,
                                               const uint8_t* __restrict__ L, const uint32_t* __restrict__ n_rows,
                                               const uint32_t* __restrict__ cnt, uint32_t* __restrict__ FL) {
  __shared__ uint32_t wb[FL_NW][256];  // per wave: the next row of each byte
  __shared__ __align__(16) uint8_t stage[FL_NW][FL_BATCH];
  const uint32_t tid = threadIdx.x, w = tid / BZG_WAVE, ln = lane();
  const uint64_t total = off[nb];
  for (uint64_t j = blockIdx.x; j < total; j += gridDim.x) {
    const uint32_t bi = owner[j], b = bl[bi], c = (uint32_t)(j - off[bi]), n = n_rows[b];
    const uint8_t* Lb = L + blks[b].l_off;
    uint32_t* F = FL + blks[b].l_off;
    const uint32_t lo = min(n, c * FL_CH + w * FL_SUB), hi = min(n, lo + FL_SUB);
    for (uint32_t q = 0; q < FL_NW; q++) wb[q][tid] = 0;
    __syncthreads();
    fl_count(Lb, lo, hi, ln, BZG_WAVE, wb[w]);
    __syncthreads();
    {
      uint32_t run = cnt[j * 256 + tid];
      for (uint32_t q = 0; q < FL_NW; q++) {
        const uint32_t x = wb[q][tid];
        wb[q][tid] = run;
        run += x;
      }
    }
    __syncthreads();
    // this wave alone until the next barrier (its LDS rows are used in
    // program order): the column FL_BATCH bytes at a time, the next batch
    // loading while this one is ranked 64 rows a step
    uint32_t* nx = wb[w];
    uint8_t* sg = stage[w];
    uint4 ahead = lo + 16 * ln < hi ? *(const uint4*)(Lb + lo + 16 * ln) : make_uint4(0, 0, 0, 0);
    for (uint32_t k0 = lo; k0 < hi; k0 += FL_BATCH) {
      ((uint4*)sg)[ln] = ahead;
      const uint32_t k1 = k0 + FL_BATCH;
      if (k1 + 16 * ln < hi) ahead = *(const uint4*)(Lb + k1 + 16 * ln);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const uint32_t steps = min(FL_BATCH, hi - k0);
      for (uint32_t s = 0; s < steps; s += BZG_WAVE) {
        const uint32_t k = k0 + s + ln;
        const bool ok = k < hi;
        const uint32_t d = ok ? sg[s + ln] : 0u;
        const uint64_t peers = match_digit8(d, __ballot(ok));
        const uint32_t base = nx[d];
        if (ok) F[base + (uint32_t)__popcll(peers & lanemask_lt())] = k | (d << 24);
        if (ok && (uint32_t)(__ffsll((long long)peers) - 1) == ln) nx[d] = base + (uint32_t)__popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------- inverse BWT from many points

// Sampled rows of a block: every WALK_STRIDE-th row, and origPtr.
__device__ __forceinline__ uint32_t samples_of(uint32_t n, uint32_t orig) {
  const uint32_t s = (n + WALK_STRIDE - 1) / WALK_STRIDE;
  return s + (orig % WALK_STRIDE ? 1u : 0u);
}
__device__ __forceinline__ uint32_t sample_row(uint32_t s, uint32_t n, uint32_t orig) {
  const uint32_t m = (n + WALK_STRIDE - 1) / WALK_STRIDE;
  return s < m ? s * WALK_STRIDE : orig;
}
__device__ __forceinline__ bool is_sample(uint32_t row, uint32_t orig) {
  return row % WALK_STRIDE == 0 || row == orig;
}
__device__ __forceinline__ uint32_t sample_index(uint32_t row, uint32_t n, uint32_t orig) {
  return row % WALK_STRIDE == 0 ? row / WALK_STRIDE : (n + WALK_STRIDE - 1) / WALK_STRIDE;
}

constexpr uint32_t UNVISITED = 0xFFFFFFFFu;

// Walker per sampled row: follows FL until the next sampled row; records
// the steps and which sample it reached.
__device__ __forceinline__ void walk_item(uint64_t j, const DecBlk* __restrict__ blks,
                                          const uint64_t* __restrict__ s0, uint32_t nb,
                                          const uint32_t* __restrict__ bl, uint64_t total,
                                          const uint32_t* __restrict__ n_rows, const uint32_t* __restrict__ origs,
                                          const uint32_t* __restrict__ FL, uint32_t* __restrict__ nxt,
                                          uint32_t* __restrict__ steps, uint32_t* __restrict__ pos) {
  if (j >= total) return;
  const uint32_t bi = owner_of_wg(s0, nb, j), b = bl[bi];
  const uint32_t s = (uint32_t)(j - s0[bi]), n = n_rows[b], orig = origs[b];
  pos[j] = UNVISITED;
  if (n == 0 || s >= samples_of(n, orig)) return;
  const uint32_t* F = FL + blks[b].l_off;
  uint32_t row = sample_row(s, n, orig), c = 0;
  do {
    row = F[row] & 0xFFFFFFu;
    c++;
  } while (!is_sample(row, orig) && c < n);
  nxt[j] = sample_index(row, n, orig);
  steps[j] = c;
}
// Walkers in tiles of NT, persistent; each XCD walks a contiguous range of
// walkers, so a block's map is read through one L2.
__global__ __launch_bounds__(NT) void k_dec_walk(const DecBlk* __restrict__ blks, const uint64_t* __restrict__ s0,
                                                 uint32_t nb, const uint32_t* __restrict__ bl,
                                                 const uint32_t* __restrict__ n_rows,
                                                 const uint32_t* __restrict__ origs, const uint32_t* __restrict__ FL,
                                                 uint32_t* __restrict__ nxt, uint32_t* __restrict__ steps,
                                                 uint32_t* __restrict__ pos) {
  const uint64_t total = s0[nb];
  for (TileLoop it = tile_loop((uint32_t)((total + NT - 1) / NT)); it.t < it.end; it.t += it.step)
    walk_item((uint64_t)it.t * NT + threadIdx.x, blks, s0, nb, bl, total, n_rows, origs, FL, nxt, steps, pos);
}

// Per block: the chain of samples from origPtr gives every walker on it its
// output position; its length is the period of the text (the whole block
// unless the block repeats a shorter string).  The chain is cut where it
// returns to origPtr's sample and ranked by pointer jumping in LDS: each
// sample's count of text bytes from itself to the cut, doubled along the
// chain each round; a walker's position is the total minus its own count.
// Samples off the chain (other cycles of a periodic block) never reach the
// cut and stay unvisited.
constexpr uint32_t CHAIN_NT = 1024;
constexpr uint32_t CHAIN_CAP = 900000 / WALK_STRIDE + 3;  // samples of the largest block, and the cut
constexpr uint32_t CHAIN_PER = (CHAIN_CAP + CHAIN_NT - 1) / CHAIN_NT;
constexpr uint32_t CHAIN_BIG = 0x40000000u;  // a count past any block (two of them sum without wrapping)
__global__ __launch_bounds__(CHAIN_NT) void k_dec_chain(const uint64_t* __restrict__ s0, uint32_t nb,
                                                        const uint32_t* __restrict__ bl,
                                                        const uint32_t* __restrict__ n_rows,
                                                        const uint32_t* __restrict__ origs,
                                                        const uint32_t* __restrict__ nxt,
                                                        const uint32_t* __restrict__ steps, uint32_t* __restrict__ pos,
                                                        uint32_t* __restrict__ period, uint32_t* __restrict__ err) {
  __shared__ uint32_t succ[CHAIN_CAP], cnt[CHAIN_CAP];
  const uint32_t bi = blockIdx.x, b = bl[bi], tid = threadIdx.x;
  const uint32_t n = n_rows[b], orig = origs[b];
  if (n == 0) {
    if (tid == 0) period[b] = 0;
    return;
  }
  const uint32_t ns = samples_of(n, orig), s_start = sample_index(orig, n, orig);
  if (ns + 1 > CHAIN_CAP) {  // a block longer than any level allows
    if (tid == 0) {
      period[b] = 0;
      atomicOr(err, ERR_STREAM);
    }
    return;
  }
  const uint64_t base = s0[bi];
  const uint32_t cut = ns;  // the node after the chain's last sample
  for (uint32_t i = tid; i <= ns; i += CHAIN_NT) {
    if (i == cut) {
      succ[i] = cut;
      cnt[i] = 0;
    } else {
      const uint32_t x = nxt[base + i];
      // a walker that found no sample ends the chain with an impossible count
      succ[i] = x == s_start || x >= ns ? cut : x;
      cnt[i] = x >= ns ? CHAIN_BIG : min(steps[base + i], CHAIN_BIG);
    }
  }
  __syncthreads();
  uint32_t rounds = 0;
  while ((1u << rounds) < ns + 1) rounds++;
  for (uint32_t r = 0; r < rounds; r++) {
    uint32_t su[CHAIN_PER], cu[CHAIN_PER];
#pragma unroll
    for (uint32_t k = 0; k < CHAIN_PER; k++) {
      const uint32_t i = tid + k * CHAIN_NT;
      if (i <= ns) {
        const uint32_t u = succ[i];
        su[k] = succ[u];
        cu[k] = min(cnt[i] + cnt[u], CHAIN_BIG);
      }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < CHAIN_PER; k++) {
      const uint32_t i = tid + k * CHAIN_NT;
      if (i <= ns) {
        succ[i] = su[k];
        cnt[i] = cu[k];
      }
    }
    __syncthreads();
  }
  const uint32_t P = cnt[s_start];
  const bool ok = succ[s_start] == cut && P > 0 && P <= n && n % P == 0;
  for (uint32_t i = tid; i < ns; i += CHAIN_NT)
    if (succ[i] == cut) pos[base + i] = ok ? P - cnt[i] : UNVISITED;
  if (tid == 0) {
    period[b] = ok ? P : 0u;
    if (!ok) atomicOr(err, ERR_STREAM);
  }
}

// Walkers on the chain write their pieces of the text (the RLE1 bytes).
__device__ __forceinline__ void emit_item(uint64_t j, const DecBlk* __restrict__ blks,
                                          const uint64_t* __restrict__ s0, uint32_t nb,
                                          const uint32_t* __restrict__ bl, uint64_t total,
                                          const uint32_t* __restrict__ n_rows, const uint32_t* __restrict__ origs,
                                          const uint32_t* __restrict__ FL, const uint32_t* __restrict__ steps,
                                          const uint32_t* __restrict__ pos, const uint32_t* __restrict__ period,
                                          uint8_t* __restrict__ T) {
  if (j >= total) return;
  const uint32_t p0 = pos[j];
  if (p0 == UNVISITED) return;
  const uint32_t bi = owner_of_wg(s0, nb, j), b = bl[bi];
  const uint32_t s = (uint32_t)(j - s0[bi]), n = n_rows[b], orig = origs[b], per = period[b];
  if (per == 0 || p0 >= per) return;
  const uint64_t o = blks[b].l_off;
  const uint32_t* F = FL + o;
  uint8_t* Tb = T + o + p0;
  uint32_t row = sample_row(s, n, orig);
  const uint32_t c = min(steps[j], per - p0);
  // the piece's bytes in order: single bytes up to a 4-byte boundary, then
  // whole words, then the rest
  uint32_t k = 0;
  for (; k < c && ((uintptr_t)(Tb + k) & 3u); k++) {
    const uint32_t v = F[row];
    row = v & 0xFFFFFFu;
    Tb[k] = (uint8_t)(v >> 24);
  }
  for (; k + 4 <= c; k += 4) {
    uint32_t w = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; i++) {
      const uint32_t v = F[row];
      row = v & 0xFFFFFFu;
      w |= (v >> 24) << (8 * i);
    }
    *(uint32_t*)(Tb + k) = w;
  }
  for (; k < c; k++) {
    const uint32_t v = F[row];
    row = v & 0xFFFFFFu;
    Tb[k] = (uint8_t)(v >> 24);
  }
}

// The walkers as in k_dec_walk.
__global__ __launch_bounds__(NT) void k_dec_emit(const DecBlk* __restrict__ blks, const uint64_t* __restrict__ s0,
                                                 uint32_t nb, const uint32_t* __restrict__ bl,
                                                 const uint32_t* __restrict__ n_rows,
                                                 const uint32_t* __restrict__ origs, const uint32_t* __restrict__ FL,
                                                 const uint32_t* __restrict__ steps,
                                                 const uint32_t* __restrict__ pos, const uint32_t* __restrict__ period,
                                                 uint8_t* __restrict__ T) {
  const uint64_t total = s0[nb];
  for (TileLoop it = tile_loop((uint32_t)((total + NT - 1) / NT)); it.t < it.end; it.t += it.step)
    emit_item((uint64_t)it.t * NT + threadIdx.x, blks, s0, nb, bl, total, n_rows, origs, FL, steps, pos, period, T);
}

// A block that repeats a string of the period: the rest is copies.
__global__ __launch_bounds__(NT) void k_dec_repeat(const DecBlk* __restrict__ blks, const uint32_t* __restrict__ bl,
                                                   const uint32_t* __restrict__ n_rows,
                                                   const uint32_t* __restrict__ period, uint8_t* __restrict__ T) {
  const uint32_t b = bl[blockIdx.x], n = n_rows[b], p = period[b];
  if (p == 0 || p >= n) return;
  uint8_t* Tb = T + blks[b].l_off;
  for (uint32_t i = p + threadIdx.x; i < n; i += NT) Tb[i] = Tb[i % p];
}

// ------------------------------------------------ run-length decoding

// RLE1 decoding state before a byte: 0 fresh, 1..3 that many equal bytes
// just written (the last one `last`), 4 a count byte expected (it repeats
// `last`).  One step on byte x: the bytes it writes and the next state.
__device__ __forceinline__ uint32_t rle_step(uint32_t& st, uint32_t& last, uint32_t x) {
  if (st == 4) {
    st = 0;
    return x;  // x more copies of last
  }
  if (st >= 1 && x == last) {
    st++;
    return 1;
  }
  st = 1;
  last = x;
  return 1;
}

// A segment's RLE_SEG bytes as words, byte i in bits 8*(i%4) of word i/4.
// Segments start 16-byte aligned (block ranges are multiples of 32 bytes)
// and the text array is padded, so all RLE_SEG bytes are read, the ones past
// the block's end unused.
__device__ __forceinline__ void seg_words(const uint8_t* __restrict__ Tb, uint32_t (&xw)[RLE_SEG / 4]) {
#pragma unroll
  for (uint32_t q = 0; q < RLE_SEG / 16; q++) {
    const uint4 v = ((const uint4*)Tb)[q];
    xw[4 * q] = v.x;
    xw[4 * q + 1] = v.y;
    xw[4 * q + 2] = v.z;
    xw[4 * q + 3] = v.w;
  }
}

// Bytes written in order from `base` through a pending aligned word: a word
// whose bytes are all this writer's is stored whole, the partial words at
// either end byte by byte (their other bytes belong to the neighbouring
// segments' writers).
struct ByteOut {
  uint8_t* base;
  uint64_t pos = 0;
  uint32_t word = 0;
  __device__ __forceinline__ void store(uint64_t wa) {
    const uint64_t lo = (uint64_t)(uintptr_t)base;
    if (wa >= lo) {
      *(uint32_t*)(uintptr_t)wa = word;
    } else {
      for (uint64_t q = lo; q < wa + 4; q++) *(uint8_t*)(uintptr_t)q = (uint8_t)(word >> (8 * (q - wa)));
    }
    word = 0;
  }
  __device__ __forceinline__ void put(uint32_t x) {
    const uint64_t ad = (uint64_t)(uintptr_t)base + pos;
    word |= x << (8 * (ad & 3u));
    pos++;
    if (((ad + 1) & 3u) == 0) store(ad & ~3ull);
  }
  __device__ __forceinline__ void fill(uint32_t x, uint32_t k) {  // k copies of x
    while (k && (((uint64_t)(uintptr_t)base + pos) & 3u)) {
      put(x);
      k--;
    }
    const uint32_t w4 = x * 0x01010101u;
    for (; k >= 4; k -= 4) {
      *(uint32_t*)(base + pos) = w4;
      pos += 4;
    }
    for (; k; k--) put(x);
  }
  __device__ __forceinline__ void finish() {
    const uint64_t ad = (uint64_t)(uintptr_t)base + pos;
    if (!(ad & 3u)) return;
    const uint64_t wa = ad & ~3ull, lo = (uint64_t)(uintptr_t)base;
    for (uint64_t q = wa > lo ? wa : lo; q < ad; q++) *(uint8_t*)(uintptr_t)q = (uint8_t)(word >> (8 * (q - wa)));
  }
};

// Per segment of RLE_SEG text bytes, for each incoming state s (with `last`
// = the segment's first byte for s = 1..3): output bytes, outgoing state and
// last byte, packed as len | st << 32 | last << 40.
__device__ __forceinline__ void rle_summ_item(uint64_t j, const DecBlk* __restrict__ blks,
                                              const uint64_t* __restrict__ g0, uint32_t nb,
                                              const uint32_t* __restrict__ bl, uint64_t total,
                                              const uint32_t* __restrict__ n_rows,
                                              const uint32_t* __restrict__ period, const uint8_t* __restrict__ T,
                                              uint64_t* __restrict__ summ) {
  if (j >= total) return;
  const uint32_t bi = owner_of_wg(g0, nb, j), b = bl[bi];
  const uint32_t g = (uint32_t)(j - g0[bi]), n = period[b] ? n_rows[b] : 0u;
  if ((uint64_t)g * RLE_SEG >= n) return;
  const uint8_t* Tb = T + blks[b].l_off + (uint64_t)g * RLE_SEG;
  const uint32_t m = min(RLE_SEG, n - g * RLE_SEG);
  uint32_t xw[RLE_SEG / 4];
  seg_words(Tb, xw);
#pragma unroll
  for (uint32_t s = 0; s < 5; s++) {
    uint32_t st = s, last = xw[0] & 255u, len = 0;
#pragma unroll
    for (uint32_t i = 0; i < RLE_SEG; i++)
      if (i < m) len += rle_step(st, last, (xw[i / 4] >> (8 * (i % 4))) & 255u);
    summ[j * 5 + s] = (uint64_t)len | ((uint64_t)st << 32) | ((uint64_t)last << 40);
  }
}

// Per block, the segments in order: each one's incoming state (and last
// byte) and output offset within the block; the block's output length.
// A segment's effect on the decoding state (0..4): the state after it, for
// each state before it, 3 bits per state.
constexpr uint32_t MAP_ID = 0u | (1u << 3) | (2u << 6) | (3u << 9) | (4u << 12);
__device__ __forceinline__ uint32_t map_at(uint32_t m, uint32_t st) { return (m >> (3 * st)) & 7u; }
// first f, then g
__device__ __forceinline__ uint32_t map_then(uint32_t f, uint32_t g) {
  uint32_t r = 0;
#pragma unroll
  for (uint32_t st = 0; st < 5; st++) r |= map_at(g, map_at(f, st)) << (3 * st);
  return r;
}

// Segments in tiles of NT, persistent.
__global__ __launch_bounds__(NT) void k_rle_summ(const DecBlk* __restrict__ blks, const uint64_t* __restrict__ g0,
                                                 uint32_t nb, const uint32_t* __restrict__ bl,
                                                 const uint32_t* __restrict__ n_rows,
                                                 const uint32_t* __restrict__ period, const uint8_t* __restrict__ T,
                                                 uint64_t* __restrict__ summ) {
  const uint64_t total = g0[nb];
  for (TileLoop it = tile_loop((uint32_t)((total + NT - 1) / NT)); it.t < it.end; it.t += it.step)
    rle_summ_item((uint64_t)it.t * NT + threadIdx.x, blks, g0, nb, bl, total, n_rows, period, T, summ);
}

// Per block (one workgroup): each segment's incoming state and last byte and
// its output offset.  A segment's summary gives, per incoming state, the
// state it leaves and its last byte; with the next segment's first byte that
// makes a map of states, so the incoming states are an ordered scan of the
// maps (composition), and the offsets a scan of the lengths those states
// pick.  KS segments per thread, NT * KS a step.
constexpr uint32_t KS = 4;
constexpr uint32_t NWV = NT / BZG_WAVE;
__global__ __launch_bounds__(NT) void k_rle_chain(const DecBlk* __restrict__ blks, const uint64_t* __restrict__ g0,
                                                  uint32_t nb, const uint32_t* __restrict__ bl,
                                                  const uint32_t* __restrict__ n_rows,
                                                  const uint32_t* __restrict__ period, const uint8_t* __restrict__ T,
                                                  const uint64_t* __restrict__ summ, uint32_t* __restrict__ seg_in,
                                                  uint32_t* __restrict__ seg_off, uint32_t* __restrict__ out_len) {
  __shared__ uint32_t wmap[NWV], wsum[NWV + 1], lastlo[NT];
  const uint32_t bi = blockIdx.x, b = bl[bi], tid = threadIdx.x, w = tid / BZG_WAVE, ln = lane();
  const uint32_t n = period[b] ? n_rows[b] : 0u;
  const uint32_t ns = (n + RLE_SEG - 1) / RLE_SEG;
  const uint8_t* Tb = T + blks[b].l_off;
  const uint64_t base = g0[bi];
  uint32_t st0 = 0, last0 = 0, off0 = 0;  // entering the step (workgroup-uniform)
  for (uint32_t t0 = 0; t0 < ns; t0 += NT * KS) {
    const uint32_t gs = t0 + tid * KS;
    uint64_t v[KS][5];
    uint32_t fm[KS];
#pragma unroll
    for (uint32_t k = 0; k < KS; k++) {
      const uint32_t g = min(gs + k, ns - 1u);
#pragma unroll
      for (uint32_t q = 0; q < 5; q++) v[k][q] = summ[(base + g) * 5 + q];
    }
    uint32_t F = MAP_ID;
#pragma unroll
    for (uint32_t k = 0; k < KS; k++) {
      const uint32_t g = gs + k;
      const uint32_t x0 = g + 1 < ns ? Tb[(g + 1) * RLE_SEG] : 0u;
      uint32_t m = 0;
#pragma unroll
      for (uint32_t q = 0; q < 5; q++) {
        const uint32_t so = (uint32_t)(v[k][q] >> 32) & 255u, lo = (uint32_t)(v[k][q] >> 40) & 255u;
        m |= ((so >= 1 && so <= 3) ? (lo == x0 ? so : 0u) : so) << (3 * q);
      }
      fm[k] = g < ns ? m : MAP_ID;
      F = map_then(F, fm[k]);
    }
    // ordered scan of the threads' maps: in the wave, then over the waves
    const uint32_t inc = wave_incl_scan(F, MAP_ID, [](uint32_t cur, uint32_t lower) { return map_then(lower, cur); });
    if (ln == BZG_WAVE - 1) wmap[w] = inc;
    __syncthreads();
    uint32_t pw = MAP_ID;
    for (uint32_t q = 0; q < w; q++) pw = map_then(pw, wmap[q]);
    const uint32_t lower = (uint32_t)__shfl_up((int)inc, 1, BZG_WAVE);
    const uint32_t ex = map_then(pw, ln == 0 ? MAP_ID : lower);  // the step's threads before this one
    uint32_t all = MAP_ID;
    for (uint32_t q = 0; q < NWV; q++) all = map_then(all, wmap[q]);
    // this thread's segments: states, lengths, last bytes
    uint32_t st = map_at(ex, st0), len = 0, my_last = 0;
    uint32_t sts[KS], lens[KS], los[KS];
#pragma unroll
    for (uint32_t k = 0; k < KS; k++) {
      const uint64_t vv = v[k][min(st, 4u)];
      sts[k] = st;
      lens[k] = gs + k < ns ? (uint32_t)vv : 0u;
      los[k] = (uint32_t)(vv >> 40) & 255u;
      len += lens[k];
      if (gs + k < ns) my_last = los[k];
      st = map_at(fm[k], st);
    }
    lastlo[tid] = my_last;
    uint32_t tot;
    const uint32_t off = block_excl_sum<uint32_t, NT>(len, wsum, &tot);  // (its barriers also order lastlo)
    uint32_t last_in = tid == 0 ? last0 : lastlo[tid - 1];
    uint32_t o = off0 + off;
#pragma unroll
    for (uint32_t k = 0; k < KS; k++) {
      const uint32_t g = gs + k;
      if (g < ns) {
        seg_in[base + g] = sts[k] | (last_in << 8);
        seg_off[base + g] = o;
      }
      o += lens[k];
      last_in = los[k];
    }
    // into the next step
    const uint32_t last_t = min(ns - t0, NT * KS) - 1u;  // the step's last segment, relative
    const uint32_t st_next = map_at(all, st0);
    const uint32_t lo_next = lastlo[last_t / KS];
    __syncthreads();
    st0 = st_next;
    last0 = lo_next;
    off0 += tot;
  }
  if (tid == 0) out_len[b] = off0;
}

// Block output offsets (one workgroup) and the total; when the total does
// not fit out_cap, every block is emptied (nothing is written) and the
// capacity error is flagged.
__global__ __launch_bounds__(1024) void k_rle_offsets(const uint32_t* __restrict__ out_len, uint32_t nb,
                                                      uint64_t out_cap, uint64_t* __restrict__ out_off,
                                                      uint64_t* __restrict__ out_bytes, uint32_t* __restrict__ skip,
                                                      uint32_t* __restrict__ err) {
  __shared__ uint64_t sh[1024 / BZG_WAVE + 1];
  const uint32_t per = (nb + 1023) / 1024, lo = min(threadIdx.x * per, nb), hi = min(lo + per, nb);
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; i++) s += out_len[i];
  uint64_t tot;
  uint64_t run = block_excl_sum<uint64_t, 1024>(s, sh, &tot);
  const bool fits = tot <= out_cap;
  for (uint32_t i = lo; i < hi; i++) {
    out_off[i] = fits ? run : 0u;
    run += out_len[i];
  }
  if (threadIdx.x == 0) {
    out_off[nb] = fits ? tot : 0u;
    *out_bytes = tot;
    *skip = fits ? 0u : 1u;
    if (!fits) atomicOr(err, ERR_CAPACITY);
  }
}

// Every segment expands its bytes at its offset (Figure 2's scatter).
__device__ __forceinline__ void rle_emit_item(uint64_t j, const DecBlk* __restrict__ blks,
                                              const uint64_t* __restrict__ g0, uint32_t nb,
                                              const uint32_t* __restrict__ bl, uint64_t total,
                                              const uint32_t* __restrict__ n_rows,
                                              const uint32_t* __restrict__ period, const uint8_t* __restrict__ T,
                                              const uint32_t* __restrict__ seg_in,
                                              const uint32_t* __restrict__ seg_off,
                                              const uint64_t* __restrict__ out_off, uint8_t* __restrict__ out) {
  if (j >= total) return;
  const uint32_t bi = owner_of_wg(g0, nb, j), b = bl[bi];
  const uint32_t g = (uint32_t)(j - g0[bi]), n = period[b] ? n_rows[b] : 0u;
  if ((uint64_t)g * RLE_SEG >= n) return;
  const uint8_t* Tb = T + blks[b].l_off + (uint64_t)g * RLE_SEG;
  const uint32_t m = min(RLE_SEG, n - g * RLE_SEG);
  uint32_t xw[RLE_SEG / 4];
  seg_words(Tb, xw);
  ByteOut o{out + out_off[b] + seg_off[j]};
  uint32_t st = seg_in[j] & 255u, last = seg_in[j] >> 8;
#pragma unroll
  for (uint32_t i = 0; i < RLE_SEG; i++) {
    if (i >= m) break;
    const uint32_t x = (xw[i / 4] >> (8 * (i % 4))) & 255u;
    if (st == 4) o.fill(last, x);
    else o.put(x);
    (void)rle_step(st, last, x);
  }
  o.finish();
}

// Segments as in k_rle_summ (nothing when the output did not fit).
__global__ __launch_bounds__(NT) void k_rle_emit(const DecBlk* __restrict__ blks, const uint64_t* __restrict__ g0,
                                                 uint32_t nb, const uint32_t* __restrict__ bl,
                                                 const uint32_t* __restrict__ n_rows,
                                                 const uint32_t* __restrict__ period, const uint8_t* __restrict__ T,
                                                 const uint32_t* __restrict__ seg_in,
                                                 const uint32_t* __restrict__ seg_off,
                                                 const uint64_t* __restrict__ out_off,
                                                 const uint32_t* __restrict__ skip, uint8_t* __restrict__ out) {
  if (*skip) return;
  const uint64_t total = g0[nb];
  for (TileLoop it = tile_loop((uint32_t)((total + NT - 1) / NT)); it.t < it.end; it.t += it.step)
    rle_emit_item((uint64_t)it.t * NT + threadIdx.x, blks, g0, nb, bl, total, n_rows, period, T, seg_in, seg_off,
                  out_off, out);
}

// Work items per block of each kind, planned on the device once the blocks'
// lengths are known (their offsets are then a scan, k_scan_counts).  None
// exceeds the bound the host sized its arrays for from the block's capacity.
enum DecPlan : int { PLAN_MTF = 0, PLAN_FL = 1, PLAN_WALK = 2, PLAN_RLE = 3 };
__global__ void k_dec_plan(int kind, uint32_t nb, const uint32_t* __restrict__ bl, const uint32_t* __restrict__ n_syms,
                           const uint32_t* __restrict__ n_rows, const uint32_t* __restrict__ origs,
                           const uint32_t* __restrict__ period, uint32_t* __restrict__ cnt) {
  const uint32_t bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= nb) return;
  const uint32_t b = bl[bi];
  uint32_t c;
  if (kind == PLAN_MTF) {
    c = (n_syms[b] + MTF_CH - 1) / MTF_CH;
  } else if (kind == PLAN_FL) {
    c = (n_rows[b] + FL_CH - 1) / FL_CH;
  } else if (kind == PLAN_WALK) {
    c = n_rows[b] ? samples_of(n_rows[b], origs[b]) : 0u;
  } else {
    const uint32_t n = period[b] ? n_rows[b] : 0u;
    c = (n + RLE_SEG - 1) / RLE_SEG;
  }
  cnt[bi] = c;
}

// Block CRCs against the stored ones, and every stream's combined CRC.
__global__ void k_dec_check(uint32_t nb, const uint32_t* __restrict__ crc_got, const uint32_t* __restrict__ crc_want,
                            uint32_t n_streams, const uint32_t* __restrict__ stream_b0,
                            const uint32_t* __restrict__ stream_crc, const uint32_t* __restrict__ skip,
                            uint32_t* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (*skip) return;
  if (i < nb && crc_got[i] != crc_want[i]) atomicOr(err, ERR_STREAM);
  if (i < n_streams) {
    uint32_t comb = 0;
    for (uint32_t k = stream_b0[i]; k < stream_b0[i + 1]; k++) comb = ((comb << 1) | (comb >> 31)) ^ crc_want[k];
    if (comb != stream_crc[i]) atomicOr(err, ERR_STREAM);
  }
}

// ------------------------------------------------------------ launchers

hipError_t dec_find(const uint8_t* in, uint64_t n, int pass, uint32_t* tile_cnt, const uint64_t* tile_off,
                    uint64_t* cand, uint64_t cand_cap, hipStream_t st) {
  const uint64_t tiles = (n + FIND_TILE - 1) / FIND_TILE;
  ProfScope ps("dec_find", st, (double)n);
  hipLaunchKernelGGL(k_find_markers, dim3((uint32_t)std::max<uint64_t>(tiles, 1)), dim3(NT), 0, st, in, n, pass,
                     tile_cnt, tile_off, cand, cand_cap);
  return hipGetLastError();
}
uint64_t dec_find_tiles(uint64_t n) { return std::max<uint64_t>((n + FIND_TILE - 1) / FIND_TILE, 1); }

hipError_t dec_scan_counts(const uint32_t* cnt, uint32_t n, uint64_t* off, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, n, off);
  return hipGetLastError();
}

uint32_t dec_walk_slots(uint32_t cap) { return cap / WALK_STRIDE + 2; }
uint32_t dec_rle_slots(uint32_t cap) { return cap / RLE_SEG + 1; }
uint32_t dec_mtf_chunks(uint32_t cap) { return cap / MTF_CH + 1; }
uint32_t dec_fl_chunks(uint32_t cap) { return cap / FL_CH + 1; }

hipError_t dec_run(const DecRun& d, hipStream_t st) {
  const uint32_t nb = d.nb;
  // per-block work items of a kind, from the lengths decoded so far
  auto plan = [&](int kind, uint64_t* off) {
    hipLaunchKernelGGL(k_dec_plan, dim3((nb + 255) / 256), dim3(256), 0, st, kind, nb, d.order, d.n_syms, d.n_rows,
                       d.orig, d.period, d.plan_cnt);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, d.plan_cnt, nb, off);
  };
  // one tile of NT items per workgroup, over the items' bound: the items
  // that exist come first in every XCD's range (the hardware hands tiles out
  // as workgroups finish, which balances walks of uneven length), and
  // workgroups past them end at once
  auto grid = [](uint64_t bound_items) { return persist_grid((bound_items + NT - 1) / NT, ONE_TILE_EACH); };
  {
    ProfScope ps("dec_block", st, 0.0);
    hipLaunchKernelGGL(k_dec_block, dim3(nb), dim3(BZG_WAVE), 0, st, d.in, d.n_in, d.blks, d.order, d.FL, d.n_syms,
                       d.mtf0, d.orig, d.crc_want, d.err);
  }
  const uint32_t gc = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(d.ch_total, 1), 1u << 16);
  {
    ProfScope ps("dec_mtf", st, 0.0);
    plan(PLAN_MTF, d.ch0);
    hipLaunchKernelGGL(k_dec_mtf_perm, dim3(gc), dim3(BZG_WAVE), 0, st, d.blks, d.ch0, nb, d.order, d.FL, d.n_syms,
                       d.T, d.cs, d.ce, d.clen, d.err);
    hipLaunchKernelGGL(k_dec_mtf_scan, dim3(nb), dim3(BZG_WAVE), 0, st, d.blks, d.ch0, d.order, d.n_syms, d.mtf0, d.T,
                       d.clen, d.coff, d.orig, d.n_rows, d.err);
    hipLaunchKernelGGL(k_dec_mtf_emit, dim3(gc), dim3(BZG_WAVE), 0, st, d.blks, d.ch0, nb, d.order, d.FL, d.n_syms,
                       d.T, d.cs, d.ce, d.coff, d.n_rows, d.L);
  }
  {
    ProfScope ps("dec_fl", st, 0.0);
    plan(PLAN_FL, d.fl_off);
    hipLaunchKernelGGL(k_dec_fl_owner, dim3((nb + 255) / 256), dim3(256), 0, st, d.fl_off, nb, d.fl_owner);
    const uint32_t gf = std::min<uint32_t>((uint32_t)std::max<uint64_t>(d.fl_total, 1),
                                           resident_grid((const void*)k_dec_fl, NT));
    hipLaunchKernelGGL(k_dec_fl_count, dim3(gf), dim3(NT), 0, st, d.blks, nb, d.order, d.fl_off, d.fl_owner, d.L,
                       d.n_rows, d.fl_cnt);
    hipLaunchKernelGGL(k_dec_fl_scan, dim3(nb), dim3(NT), 0, st, d.fl_off, d.fl_cnt);
    hipLaunchKernelGGL(k_dec_fl, dim3(gf), dim3(NT), 0, st, d.blks, nb, d.order, d.fl_off, d.fl_owner, d.L, d.n_rows,
                       d.fl_cnt, d.FL);
  }
  const uint32_t gw = grid(d.walk_total);
  const uint32_t ge = grid(d.walk_total);
  {
    ProfScope ps("dec_walk", st, 0.0);
    plan(PLAN_WALK, d.walk0);
    hipLaunchKernelGGL(k_dec_walk, dim3(gw), dim3(NT), 0, st, d.blks, d.walk0, nb, d.order, d.n_rows, d.orig, d.FL,
                       d.nxt, d.steps, d.pos);
  }
  hipLaunchKernelGGL(k_dec_chain, dim3(nb), dim3(CHAIN_NT), 0, st, d.walk0, nb, d.order, d.n_rows, d.orig, d.nxt,
                     d.steps, d.pos, d.period, d.err);
  {
    ProfScope ps("dec_emit", st, 0.0);
    hipLaunchKernelGGL(k_dec_emit, dim3(ge), dim3(NT), 0, st, d.blks, d.walk0, nb, d.order, d.n_rows, d.orig, d.FL,
                       d.steps, d.pos, d.period, d.T);
  }
  hipLaunchKernelGGL(k_dec_repeat, dim3(nb), dim3(NT), 0, st, d.blks, d.order, d.n_rows, d.period, d.T);
  const uint32_t gs = grid(d.rle_total);
  {
    ProfScope ps("dec_rle", st, 0.0);
    plan(PLAN_RLE, d.rle0);
    hipLaunchKernelGGL(k_rle_summ, dim3(gs), dim3(NT), 0, st, d.blks, d.rle0, nb, d.order, d.n_rows, d.period, d.T,
                       d.summ);
    hipLaunchKernelGGL(k_rle_chain, dim3(nb), dim3(NT), 0, st, d.blks, d.rle0, nb, d.order, d.n_rows, d.period, d.T,
                       d.summ, d.seg_in, d.seg_off, d.out_len);
  }
  return hipGetLastError();
}

// The output offsets of all blocks, in stream order (once every class has
// its blocks' lengths).
hipError_t dec_offsets(const DecRun& d, uint32_t nb, hipStream_t st) {
  ProfScope ps("dec_rle", st, 0.0);
  hipLaunchKernelGGL(k_rle_offsets, dim3(1), dim3(1024), 0, st, d.out_len, nb, d.out_cap, d.out_off, d.out_bytes,
                     d.skip, d.err);
  return hipGetLastError();
}

// A class's output: its run-length segments expanded at their offsets.
hipError_t dec_output(const DecRun& d, hipStream_t st) {
  const uint32_t nb = d.nb;
  const uint32_t gr = persist_grid((d.rle_total + NT - 1) / NT, ONE_TILE_EACH);
  ProfScope ps("dec_rle", st, 0.0);
  hipLaunchKernelGGL(k_rle_emit, dim3(gr), dim3(NT), 0, st, d.blks, d.rle0, nb, d.order, d.n_rows, d.period, d.T,
                     d.seg_in, d.seg_off, d.out_off, d.skip, d.out);
  return hipGetLastError();
}

hipError_t dec_check(uint32_t nb, const uint32_t* crc_got, const uint32_t* crc_want, uint32_t n_streams,
                     const uint32_t* stream_b0, const uint32_t* stream_crc, const uint32_t* skip, uint32_t* err,
                     hipStream_t st) {
  const uint32_t n = std::max(nb, n_streams);
  hipLaunchKernelGGL(k_dec_check, dim3((n + 255) / 256 + 1), dim3(256), 0, st, nb, crc_got, crc_want, n_streams,
                     stream_b0, stream_crc, skip, err);
  return hipGetLastError();
}

}  // namespace bzg
