// Huffman code tables per block (Sec. 3.4: Huffman coding; Sec. 4: tables
// chosen by analysing the data).  The paper gives no GPU tree construction
// and deems one unlikely; the table choice is spread over kernels instead:
//
//  setup   table count G from the symbol count; an equal-frequency partition
//          of the alphabet gives the starting tables (cost 0 inside a table's
//          range, 15 outside).
//  assign  (tile-parallel, many workgroups per block) every 50-symbol group
//          picks the table with the least total code length, lowest index on
//          ties, and its symbols are counted for that table.  Costs come from
//          one 64-bit word per symbol holding six 10-bit lengths, so a group's
//          six costs are one sum of 50 words.
//  build   (one wave per table) textbook Huffman on (weight, id) keys with
//          weights floored at 1: the wave ranks the leaves, one lane runs the
//          two-queue merge (leaves in key order, internal nodes in creation
//          order -- their weights never decrease, so each queue head is its
//          queue's minimum), every lane walks its leaves to the root; lengths
//          over 17 halve the weights (w -> 1 + w/2) and rebuild.
//  assign and build run four times; then per-group data bits under the final
//  tables, canonical codes in (length, symbol) order, and the selectors' MTF
//  indices (list 0..G-1) from a prefix-max of each table's last use.
#include <climits>

#include "common.hpp"
#include "internal.hpp"

namespace bzg {

constexpr uint32_t ASSIGN_GROUPS = 512;      // selector groups per assign tile (large calls)
constexpr uint32_t ASSIGN_GROUPS_SMALL = 128;  // ... for calls that would not fill the GPU with 512
constexpr uint32_t ASSIGN_SUB = NT;          // groups staged in LDS at a time
constexpr uint32_t ASSIGN_SYMS = ASSIGN_SUB * GROUP;
constexpr uint32_t SEL_CHUNK = 18432;        // selectors staged in LDS at a time

struct HuffScratch {
  uint32_t w[MAXA];
  uint32_t key[MAXA];  // (weight << 9) | id
  uint32_t lw[MAXA];   // leaf weights in key order
  uint16_t order[MAXA];
  uint32_t ids2[MAXA];  // order[i] | order[min(i + 1, a - 1)] << 16: both leaf heads in one read
  uint16_t parent[2 * MAXA];
};

// One wave, one Huffman pass over the weights hs->w[0..a): ranks the leaves
// by (weight, id) and runs the two-queue merge; parents are left in
// hs->parent.  All 64 lanes call it.
__device__ void huff_pass_wave(int a, HuffScratch* hs) {
  const int l = (int)lane();
  // (weight, id) as one unique key: weights are symbol counts < 2^22
  for (int i = l; i < a; i += 64) hs->key[i] = (hs->w[i] << 9) | (uint32_t)i;
  __builtin_amdgcn_wave_barrier();
  {
    uint32_t k[5], r[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
      k[q] = (q * 64 + l < a) ? hs->key[q * 64 + l] : 0xFFFFFFFFu;
      r[q] = 0;
    }
    int j = 0;
    for (; j + 4 <= a; j += 4) {
      const uint32_t k0 = hs->key[j], k1 = hs->key[j + 1], k2 = hs->key[j + 2], k3 = hs->key[j + 3];
#pragma unroll
      for (int q = 0; q < 5; q++)
        r[q] += (uint32_t)(k0 < k[q]) + (uint32_t)(k1 < k[q]) + (uint32_t)(k2 < k[q]) + (uint32_t)(k3 < k[q]);
    }
    for (; j < a; j++) {
      const uint32_t kj = hs->key[j];
#pragma unroll
      for (int q = 0; q < 5; q++) r[q] += (uint32_t)(kj < k[q]);
    }
#pragma unroll
    for (int q = 0; q < 5; q++) {
      if (q * 64 + l < a) {
        hs->order[r[q]] = (uint16_t)(q * 64 + l);
        hs->lw[r[q]] = k[q] >> 9;
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  for (int i = l; i < a; i += 64) hs->ids2[i] = (uint32_t)hs->order[i] | ((uint32_t)hs->order[min(i + 1, a - 1)] << 16);
  __builtin_amdgcn_wave_barrier();
  // Two-queue merge: leaves by (weight, id) in hs->lw / hs->order, internal
  // nodes in creation order (their weights never decrease) in hs->w (free
  // after the ranking).  Each step reads both heads of both queues in one
  // batch of LDS reads (clamped indices, empty queues read as infinite) and
  // picks the two smallest with selects, leaves first on ties.  Lane 0
  // writes; all lanes read the same words.  Depths are left to the walk.
  uint32_t* const wn = hs->w;
  const uint32_t A_ = (uint32_t)a, INF = 0xFFFFFFFFu;
  uint32_t li = 0, ni = 0, nn = 0;
  for (uint32_t step = 0; step + 1 < A_; step++) {
    const uint32_t l0 = min(li, A_ - 1u), l1 = min(li + 1u, A_ - 1u);
    const uint32_t n0 = min(ni, A_ - 2u), n1 = min(ni + 1u, A_ - 2u);
    const uint32_t lwa = hs->lw[l0], lwb = hs->lw[l1];
    const uint32_t ids = hs->ids2[l0];  // order[l0] and order[l1] (l1 = min(l0 + 1, A_ - 1))
    const uint32_t wna = wn[n0], wnb = wn[n1];
    // ids is used only by lane 0's writes: without this the compiler moves
    // its read into that branch and waits for it there, a second round trip
    asm volatile("" ::"v"(ids));
    const uint32_t ida = ids & 0xFFFFu, idb = ids >> 16;
    const uint32_t A0 = li < A_ ? lwa : INF, A1 = li + 1u < A_ ? lwb : INF;
    const uint32_t B0 = ni < nn ? wna : INF, B1 = ni + 1u < nn ? wnb : INF;
    const bool p1 = A0 <= B0;  // first pick is a leaf
    const uint32_t C = p1 ? A1 : A0, D = p1 ? B0 : B1;
    const bool p2 = C <= D;    // second pick is a leaf
    const uint32_t w1 = p1 ? A0 : B0, w2 = p2 ? C : D;
    const uint32_t id1 = p1 ? ida : A_ + ni;
    const uint32_t id2 = p2 ? (p1 ? idb : ida) : (p1 ? A_ + ni : A_ + ni + 1u);
    if (l == 0) {
      hs->parent[id1] = (uint16_t)(A_ + nn);
      hs->parent[id2] = (uint16_t)(A_ + nn);
      wn[nn] = w1 + w2;
    }
    const uint32_t nl = (p1 ? 1u : 0u) + (p2 ? 1u : 0u);
    li += nl;
    ni += 2u - nl;
    nn++;
  }
  __builtin_amdgcn_wave_barrier();
}

// One wave: leaf depths from the parents of the last pass (leaf 64*q + lane
// in dep[q]); returns the deepest.
constexpr int WALK_COLS = (MAXA + 63) / 64;
__device__ uint32_t huff_walk_wave(int a, const HuffScratch* hs, uint32_t dep[WALK_COLS]) {
  const int root = 2 * a - 2;
  uint32_t dmax = 0;
#pragma unroll
  for (int q = 0; q < WALK_COLS; q++) {
    const int i = q * 64 + (int)lane();
    int d = 0, v = i;
    while (i < a && v != root && d < 2 * MAXA) {  // parents have larger ids: at most 2a steps
      v = hs->parent[v];
      d++;
    }
    dep[q] = (uint32_t)d;
    dmax = max(dmax, (uint32_t)d);
  }
  return wave_max(dmax);
}

__device__ __forceinline__ int n_tables(uint32_t ns, int a) {
  int g = ns < 200 ? 2 : ns < 600 ? 3 : ns < 1200 ? 4 : ns < 2400 ? 5 : 6;
  return g < a ? g : a;
}

__device__ __forceinline__ uint64_t pack_costs(const BlockTables* T, int G, int v) {
  uint64_t c = 0;
  for (int t = 0; t < G; t++) c |= (uint64_t)T->len[t][v] << (10 * t);
  return c;
}

// Per block: sizes, the starting tables, cleared counters, and zero data
// bits for the block's group slots past its last group (the slots the final
// assign pass does not write; the last block also clears the end slot).
__global__ __launch_bounds__(NT) void k_huff_setup(const uint32_t* __restrict__ nsyms, const uint32_t* __restrict__ freq,
                                                   const uint32_t* __restrict__ inuse, BlockTables* __restrict__ tabs,
                                                   uint64_t* __restrict__ cost, uint32_t* __restrict__ tf,
                                                   const uint64_t* __restrict__ sel_base, uint64_t* __restrict__ gbits) {
  __shared__ uint32_t sf[MAXA];
  __shared__ int rng[MAXG][2];
  const uint32_t b = blockIdx.x;
  BlockTables* T = &tabs[b];
  uint32_t nu = 0;
  for (int j = 0; j < 8; j++) nu += __popc(inuse[b * 8 + j]);
  const int a = (int)nu + 2;
  const uint32_t ns = nsyms[b];
  const int G = ns ? n_tables(ns, a) : 0;  // an empty block gets no tables and no bits
  {
    const uint64_t gb0 = sel_base[b] + (ns + GROUP - 1) / GROUP, gb1 = sel_base[b + 1];
    for (uint64_t g = gb0 + threadIdx.x; g < gb1; g += NT) gbits[g] = 0;
    if (b + 1 == gridDim.x && threadIdx.x == 0) gbits[gb1] = 0;
  }
  if (G == 0) {
    if (threadIdx.x == 0) {
      T->G = 0;
      T->nsel = 0;
      T->alpha = (uint32_t)a;
      T->data_bits = 0;
      T->hdr_bits = 0;
    }
    return;
  }
  for (int v = threadIdx.x; v < a; v += NT) sf[v] = freq[(size_t)b * MAXA + v];
  __syncthreads();
  // inclusive prefix sums of the counts (two symbols per thread): a table's
  // range sum is then a difference of two of them
  __shared__ uint32_t spre[MAXA];
  __shared__ uint32_t ssh[NT / BZG_WAVE + 1];
  static_assert(2 * NT >= MAXA, "two symbols per thread");
  {
    const int v0 = 2 * (int)threadIdx.x, v1 = v0 + 1;
    const uint32_t f0 = v0 < a ? sf[v0] : 0u, f1 = v1 < a ? sf[v1] : 0u;
    uint32_t all;
    const uint32_t ex = block_excl_sum<uint32_t, NT>(f0 + f1, ssh, &all);
    if (v0 < a) spre[v0] = ex + f0;
    if (v1 < a) spre[v1] = ex + f0 + f1;
  }
  __syncthreads();
  // The partition, one table after another: each table takes symbols from
  // gs on until its count times the tables left reaches the remaining count,
  // leaving at least one symbol per later table.  Wave 0 tests 64 candidate
  // range ends at a time and takes the first that stops.
  if (threadIdx.x < BZG_WAVE) {
    const int l = (int)lane();
    if (l == 0) {
      T->G = (uint32_t)G;
      T->nsel = (ns + GROUP - 1) / GROUP;
      T->alpha = (uint32_t)a;
      T->data_bits = 0;
    }
    uint64_t rem = ns;
    int gs = 0;
    for (int t = 0; t < G; t++) {
      const int left = G - t;
      int ge;
      uint64_t acc;
      if (left == 1) {
        ge = a - 1;
        acc = rem;
      } else {
        const uint32_t before = gs ? spre[gs - 1] : 0u;
        ge = -1;
        for (int base = gs; ge < 0; base += BZG_WAVE) {  // ends by base + 63 >= a - left
          const int v = base + l;
          const uint64_t sum = (uint64_t)(spre[min(v, a - 1)] - before);
          const uint64_t m = __ballot((v >= a - left) || (sum * (uint64_t)left >= rem));
          if (m) ge = base + (int)__ffsll((long long)m) - 1;
        }
        acc = (uint64_t)(spre[ge] - before);
      }
      if (l == 0) {
        rng[t][0] = gs;
        rng[t][1] = ge;
      }
      rem -= acc;
      gs = ge + 1;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < G * MAXA; i += NT) {
    const int t = i / MAXA, v = i % MAXA;
    if (v < a) T->len[t][v] = (v >= rng[t][0] && v <= rng[t][1]) ? 0 : 15;
  }
  for (int v = threadIdx.x; v < a; v += NT) {
    uint64_t c = 0;
    for (int t = 0; t < G; t++) c |= (uint64_t)((v >= rng[t][0] && v <= rng[t][1]) ? 0 : 15) << (10 * t);
    cost[(size_t)b * MAXA + v] = c;
  }
  for (int i = threadIdx.x; i < MAXG * MAXA; i += NT) tf[(size_t)b * MAXG * MAXA + i] = 0;
}

// Precomputed tables (Sec. 4: tables made beforehand from data, so no tree
// is built per block): block b takes the fixed_g given tables restricted to
// its alphabet -- symbols 0..a-2 as they are, EOB (a-1) with the length of
// symbol MAXA-1, the EOB of a block with every byte in use.  The selectors
// are then chosen once (k_huff_assign mode 0) and no table is rebuilt.
__global__ __launch_bounds__(NT) void k_huff_fixed_setup(const uint32_t* __restrict__ nsyms,
                                                         const uint32_t* __restrict__ inuse,
                                                         BlockTables* __restrict__ tabs, uint32_t* __restrict__ tf,
                                                         const uint64_t* __restrict__ sel_base,
                                                         uint64_t* __restrict__ gbits,
                                                         const uint8_t* __restrict__ fixed, int fixed_g) {
  const uint32_t b = blockIdx.x;
  BlockTables* T = &tabs[b];
  uint32_t nu = 0;
  for (int j = 0; j < 8; j++) nu += __popc(inuse[b * 8 + j]);
  const int a = (int)nu + 2;
  const uint32_t ns = nsyms[b];
  const int G = ns ? fixed_g : 0;
  {
    const uint64_t gb0 = sel_base[b] + (ns + GROUP - 1) / GROUP, gb1 = sel_base[b + 1];
    for (uint64_t g = gb0 + threadIdx.x; g < gb1; g += NT) gbits[g] = 0;
    if (b + 1 == gridDim.x && threadIdx.x == 0) gbits[gb1] = 0;
  }
  if (threadIdx.x == 0) {
    T->G = (uint32_t)G;
    T->nsel = G ? (ns + GROUP - 1) / GROUP : 0;
    T->alpha = (uint32_t)a;
    T->data_bits = 0;
    T->hdr_bits = 0;
  }
  for (int i = threadIdx.x; i < G * MAXA; i += NT) {
    const int t = i / MAXA, v = i % MAXA;
    if (v < a) T->len[t][v] = fixed[t * MAXA + (v == a - 1 ? MAXA - 1 : v)];
  }
  for (int i = threadIdx.x; i < MAXG * MAXA; i += NT) tf[(size_t)b * MAXG * MAXA + i] = 0;
}

// Tile of tg groups of one block.  mode 0: choose tables and count
// symbols per table; mode 1: data bits of every group under the final tables.
__device__ void huff_assign_tile(uint32_t j, int mode, const uint32_t* __restrict__ tile_blk,
                                 const uint32_t* __restrict__ blk_tile0, const uint16_t* __restrict__ syms,
                                 const uint64_t* __restrict__ sym_base, const uint32_t* __restrict__ nsyms,
                                 const uint64_t* __restrict__ sel_base, uint8_t* __restrict__ sel,
                                 const uint64_t* __restrict__ cost, uint32_t* __restrict__ tf,
                                 uint64_t* __restrict__ gbits, BlockTables* __restrict__ tabs, uint32_t tg,
                                 bool clamp_syms) {
  __shared__ uint16_t st[ASSIGN_SYMS];
  __shared__ uint64_t sc[MAXA];
  __shared__ uint32_t stf[MAXG][MAXA];
  __shared__ uint8_t slen[MAXG][MAXA];
  __shared__ uint64_t sh[NT / BZG_WAVE + 1];
  const uint32_t b = tile_blk[j];
  BlockTables* T = &tabs[b];
  const uint32_t nsel = T->nsel, G = T->G, a = T->alpha;
  const uint32_t g0 = (j - blk_tile0[b]) * tg;
  if (g0 >= nsel) return;
  const uint32_t g1 = min(g0 + tg, nsel);
  const uint32_t ns = nsyms[b];
  const uint16_t* S = syms + sym_base[b];
  const uint64_t sb = sel_base[b];
  if (mode == 0) {
    // every table's length of a symbol packed in 10-bit fields (loads of all
    // six tables issued together; unused tables masked out)
    for (uint32_t v = threadIdx.x; v < a; v += NT) {
      uint32_t lv[MAXG];
#pragma unroll
      for (int t = 0; t < MAXG; t++) lv[t] = T->len[t][v];
      uint64_t c = 0;
#pragma unroll
      for (int t = 0; t < MAXG; t++) c |= (uint32_t)t < G ? (uint64_t)lv[t] << (10 * t) : 0ull;
      sc[v] = c;
    }
    for (uint32_t i = threadIdx.x; i < MAXG * MAXA; i += NT) (&stf[0][0])[i] = 0;
  } else {
    stage_to_lds<NT, 8>(&slen[0][0], &T->len[0][0], G * MAXA);
  }
  uint64_t bits = 0;
  for (uint32_t gs = g0; gs < g1; gs += ASSIGN_SUB) {
    const uint32_t ge = min(gs + ASSIGN_SUB, g1);
    const uint32_t s0 = gs * GROUP, s1 = min(ge * GROUP, ns);
    __syncthreads();
    stage_to_lds<NT, 10>(st, S + s0, s1 - s0);
    __syncthreads();
    if (clamp_syms) {  // caller-given symbols: out-of-range ones (flagged by k_freq) stay inside the tables
      for (uint32_t i = threadIdx.x; i < s1 - s0; i += NT) st[i] = (uint16_t)min((uint32_t)st[i], (uint32_t)MAXA - 1u);
      __syncthreads();
    }
    const uint32_t g = gs + threadIdx.x;
    if (g < ge) {
      const uint32_t lo = g * GROUP - s0, hi = min(g * GROUP + GROUP, ns) - s0;
      const bool full = hi - lo == (uint32_t)GROUP;  // all but a block's last group
      if (mode == 0) {
        uint64_t acc = 0;
        if (full) {  // unrolled: the 50 lookups are independent
#pragma unroll
          for (uint32_t i = 0; i < (uint32_t)GROUP; i++) acc += sc[st[lo + i]];
        } else {
          for (uint32_t i = lo; i < hi; i++) acc += sc[st[i]];
        }
        uint32_t best = 0, bc = (uint32_t)(acc & 1023u);
        for (uint32_t t = 1; t < G; t++) {
          uint32_t c = (uint32_t)((acc >> (10 * t)) & 1023u);
          if (c < bc) {
            bc = c;
            best = t;
          }
        }
        sel[sb + g] = (uint8_t)best;
        if (full) {
#pragma unroll
          for (uint32_t i = 0; i < (uint32_t)GROUP; i++) atomicAdd(&stf[best][st[lo + i]], 1u);
        } else {
          for (uint32_t i = lo; i < hi; i++) atomicAdd(&stf[best][st[i]], 1u);
        }
      } else {
        const uint32_t t = sel[sb + g];
        uint32_t acc = 0;
        if (full) {
#pragma unroll
          for (uint32_t i = 0; i < (uint32_t)GROUP; i++) acc += slen[t][st[lo + i]];
        } else {
          for (uint32_t i = lo; i < hi; i++) acc += slen[t][st[i]];
        }
        gbits[sb + g] = acc;
        bits += acc;
      }
    }
  }
  __syncthreads();
  if (mode == 0) {
    for (uint32_t i = threadIdx.x; i < G * MAXA; i += NT) {
      uint32_t t = i / MAXA, v = i % MAXA;
      if (v < a && stf[t][v]) atomicAdd(&tf[((size_t)b * MAXG + t) * MAXA + v], stf[t][v]);
    }
  } else {
    uint64_t tot = block_sum<uint64_t, NT>(bits, sh);
    if (threadIdx.x == 0) atomicAdd((unsigned long long*)&T->data_bits, (unsigned long long)tot);
  }
}

// Persistent workgroups over the *n_tiles assign tiles (at most cap).
__global__ __launch_bounds__(NT) void k_huff_assign(int mode, const uint32_t* __restrict__ tile_blk,
                                                    const uint32_t* __restrict__ blk_tile0,
                                                    const uint16_t* __restrict__ syms,
                                                    const uint64_t* __restrict__ sym_base,
                                                    const uint32_t* __restrict__ nsyms,
                                                    const uint64_t* __restrict__ sel_base, uint8_t* __restrict__ sel,
                                                    const uint64_t* __restrict__ cost, uint32_t* __restrict__ tf,
                                                    uint64_t* __restrict__ gbits, BlockTables* __restrict__ tabs,
                                                    uint32_t tg, const uint32_t* __restrict__ n_tiles, uint32_t cap,
                                                    int clamp_syms) {
  for (TileLoop it = tile_loop(min(*n_tiles, cap)); it.t < it.end; it.t += it.step) {
    huff_assign_tile(it.t, mode, tile_blk, blk_tile0, syms, sym_base, nsyms, sel_base, sel, cost, tf, gbits, tabs, tg,
                     clamp_syms != 0);
    __syncthreads();
  }
}

// One workgroup per (block, table): new code lengths from the counts.  The
// oracle halves the weights (w -> 1 + w/2) and rebuilds until no length
// exceeds 17; here BUILD_WAVES waves try k = base .. base+7 halvings at once
// and the smallest k that fits wins -- the same k the sequential loop stops
// at.  The counts are cleared for the next pass.
constexpr int BUILD_WAVES = 1;
constexpr int BUILD_NT = BUILD_WAVES * BZG_WAVE;

__global__ __launch_bounds__(BUILD_NT) void k_huff_build(BlockTables* __restrict__ tabs, uint32_t* __restrict__ tf) {
  __shared__ uint32_t sf[MAXA];
  __shared__ HuffScratch hs[BUILD_WAVES];
  __shared__ uint32_t ok[BUILD_WAVES];
  const uint32_t b = blockIdx.x, t = blockIdx.y;
  BlockTables* T = &tabs[b];
  const int G = (int)T->G, a = (int)T->alpha;
  if ((int)t >= G) return;
  uint32_t* F = tf + ((size_t)b * MAXG + t) * MAXA;
  {
    constexpr int PF = (MAXA + BUILD_NT - 1) / BUILD_NT;
    uint32_t fv[PF];  // all loads issued before any is used (clamped index)
#pragma unroll
    for (int q = 0; q < PF; q++) fv[q] = F[min(q * BUILD_NT + (int)threadIdx.x, a - 1)];
#pragma unroll
    for (int q = 0; q < PF; q++) {
      const int i = q * BUILD_NT + (int)threadIdx.x;
      if (i < a) {
        sf[i] = fv[q];
        F[i] = 0;
      }
    }
  }
  __syncthreads();
  const int w = threadIdx.x / BZG_WAVE;
  for (int base = 0;; base += BUILD_WAVES) {
    const int k = base + w;
    for (int i = lane(); i < a; i += BZG_WAVE) {
      uint32_t x = sf[i] ? sf[i] : 1u;
      for (int r = 0; r < k && x > 2u; r++) x = 1u + x / 2u;  // 1 and 2 are fixed points
      hs[w].w[i] = x;
    }
    huff_pass_wave(a, &hs[w]);
    uint32_t dep[WALK_COLS];
    const uint32_t dmax = huff_walk_wave(a, &hs[w], dep);
    if (lane() == 0) ok[w] = dmax <= (uint32_t)MAXLEN ? 1u : 0u;
    __syncthreads();
    int first = BUILD_WAVES;
    for (int q = BUILD_WAVES - 1; q >= 0; q--)
      if (ok[q]) first = q;
    if (first < BUILD_WAVES) {
      if (w == first) {
#pragma unroll
        for (int q = 0; q < WALK_COLS; q++)
          if (q * 64 + (int)lane() < a) T->len[t][q * 64 + lane()] = (uint8_t)dep[q];
      }
      break;
    }
    __syncthreads();
  }
}

// Per block: canonical codes, selector MTF indices and header bit count.
__global__ __launch_bounds__(NT) void k_huff_finish(const uint32_t* __restrict__ inuse,
                                                    const uint64_t* __restrict__ sel_base,
                                                    const uint8_t* __restrict__ sel, uint8_t* __restrict__ selmtf,
                                                    BlockTables* __restrict__ tabs) {
  __shared__ uint8_t lens[MAXG][MAXA];
  __shared__ uint32_t s_first[MAXG][MAXLEN + 2];
  __shared__ uint32_t sh[NT / BZG_WAVE + 1];
  const uint32_t b = blockIdx.x;
  const uint32_t tid = threadIdx.x;
  BlockTables* T = &tabs[b];
  const int G = (int)T->G, a = (int)T->alpha;
  if (G == 0) return;  // empty block: nothing to code, hdr_bits stays 0
  const uint32_t nsel = T->nsel;
  const uint64_t sb = sel_base[b];
  __shared__ uint32_t lcnt[MAXG][MAXLEN + 2];
  for (uint32_t i = tid; i < MAXG * (MAXLEN + 2); i += NT) (&lcnt[0][0])[i] = 0;
  stage_to_lds<NT, 8>(&lens[0][0], &T->len[0][0], (uint32_t)(G * MAXA));
  __syncthreads();
  // canonical codes: per table, the first code of every length
  for (int i = tid; i < G * MAXA; i += NT) {
    const int t = i / MAXA, v = i % MAXA;
    if (v < a) atomicAdd(&lcnt[t][lens[t][v]], 1u);
  }
  __syncthreads();
  if (tid < (uint32_t)G) {
    uint32_t code = 0;
    for (int q = 1; q <= MAXLEN; q++) {
      s_first[tid][q] = code;
      code = (code + lcnt[tid][q]) << 1;
    }
  }
  __syncthreads();
  // code = the first code of its length + its rank among the table's
  // symbols of that length, in symbol order.  One wave per table, 64 symbols
  // at a time: lanes of equal length are found by ballots, and a per-length
  // running count (LDS, this wave's own) carries the ranks across the rounds.
  {
    __shared__ uint32_t srun[NT / BZG_WAVE][MAXLEN + 2];
    const int w = (int)(tid / BZG_WAVE);
    const uint64_t lt = lanemask_lt();
    for (int t = w; t < G; t += NT / BZG_WAVE) {
      if (lane() < MAXLEN + 2) srun[w][lane()] = 0;
      for (int k = 0; k * BZG_WAVE < a; k++) {
        const int v = k * BZG_WAVE + (int)lane();
        const bool ok = v < a;
        const uint32_t L = ok ? lens[t][v] : 0u;
        const uint64_t peers = match_digit8(L, __ballot(ok));
        const uint32_t before = srun[w][L];
        if (ok) T->code[t][v] = s_first[t][L] + before + (uint32_t)__popcll(peers & lt);
        // the lowest lane of each length adds the round's count (the wave's
        // LDS operations complete in order: every lane has read first)
        if (ok && (uint32_t)(__ffsll((long long)peers) - 1) == lane()) srun[w][L] = before + (uint32_t)__popcll(peers);
      }
    }
  }
  // selector MTF indices, SEL_CHUNK selectors at a time staged in LDS:
  // thread-contiguous ranges; a table's rank in the list at a selector is the
  // number of tables used more recently, so each thread starts from the
  // prefix-max of last uses before its range (carried across chunks).  The
  // per-table arrays are indexed by unrolled loops only (no lane-varying
  // register index).
  __shared__ uint8_t ssel[SEL_CHUNK];
  __shared__ int swl[NT / BZG_WAVE][MAXG];
  const int w = (int)(tid / BZG_WAVE);
  int carry[MAXG];
#pragma unroll
  for (int v = 0; v < MAXG; v++) carry[v] = -1 - v;  // initial list 0..G-1, 0 most recent
  uint32_t sbits = 0;
  for (uint32_t c0 = 0; c0 < nsel; c0 += SEL_CHUNK) {
    const uint32_t cn = min(SEL_CHUNK, nsel - c0);
    __syncthreads();
    stage_to_lds<NT, 8>(ssel, sel + sb + c0, cn);
    __syncthreads();
    const uint32_t per = (cn + NT - 1) / NT;
    const uint32_t g0 = min(tid * per, cn), g1 = min(g0 + per, cn);
    int loc[MAXG], lastv[MAXG];
#pragma unroll
    for (int v = 0; v < MAXG; v++) loc[v] = INT_MIN;
    for (uint32_t g = g0; g < g1; g++) {
      const int x = ssel[g];
#pragma unroll
      for (int v = 0; v < MAXG; v++) loc[v] = x == v ? (int)(c0 + g) : loc[v];
    }
    // one workgroup prefix-max of all tables' last uses
#pragma unroll
    for (int v = 0; v < MAXG; v++) loc[v] = wave_incl_max(loc[v]);
    if (lane() == BZG_WAVE - 1) {
#pragma unroll
      for (int v = 0; v < MAXG; v++) swl[w][v] = loc[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < MAXG; v++) {
      int before = INT_MIN, all = INT_MIN;
      for (int q = 0; q < NT / BZG_WAVE; q++) {
        before = q < w ? max(before, swl[q][v]) : before;
        all = max(all, swl[q][v]);
      }
      const int up = wave_shr1(INT_MIN, loc[v]);  // lane 0: none before it
      lastv[v] = max(carry[v], max(before, up));
      carry[v] = max(carry[v], all);
    }
    for (uint32_t g = g0; g < g1; g++) {
      const int x = ssel[g];
      int lx = 0;
#pragma unroll
      for (int v = 0; v < MAXG; v++) lx = x == v ? lastv[v] : lx;
      uint32_t idx = 0;
#pragma unroll
      for (int v = 0; v < MAXG; v++) idx += (v < G && v != x && lastv[v] > lx) ? 1u : 0u;
      ssel[g] = (uint8_t)idx;  // only this thread reads position g
#pragma unroll
      for (int v = 0; v < MAXG; v++) lastv[v] = x == v ? (int)(c0 + g) : lastv[v];
      sbits += idx + 1;
    }
    __syncthreads();
    for (uint32_t i = tid; i < cn; i += NT) selmtf[sb + c0 + i] = ssel[i];
  }
  // delta-coded lengths: 2|d| + 1 bits per symbol, 5 per table
  for (int i = tid; i < G * MAXA; i += NT) {
    const int t = i / MAXA, v = i % MAXA;
    if (v < a) {
      const int d = (int)lens[t][v] - (int)lens[t][v ? v - 1 : 0];
      sbits += 2u * (uint32_t)(d < 0 ? -d : d) + 1u;
    }
  }
  uint32_t stot = block_sum<uint32_t, NT>(sbits, sh);
  if (tid == 0) {
    uint32_t ranges = 0;
    for (int j = 0; j < 8; j++) {
      uint32_t x = inuse[b * 8 + j];
      ranges += ((x & 0xFFFFu) ? 1u : 0u) + ((x >> 16) ? 1u : 0u);
    }
    T->hdr_bits = 16 + 16 * ranges + 3 + 15 + stot + 5u * (uint32_t)G;
  }
}

// Per-block symbol histogram (for callers that pass symbols directly).  The
// block's count is clamped to its capacity and stored in ns_out; a symbol
// outside the block's alphabet (in-use bytes + 2), or a count above the
// capacity, sets ERR_SYMBOL.
__global__ __launch_bounds__(NT) void k_freq(const uint16_t* __restrict__ syms, const uint64_t* __restrict__ sym_off,
                                             const uint32_t* __restrict__ nsyms, const uint32_t* __restrict__ inuse,
                                             uint32_t* __restrict__ freq, uint32_t* __restrict__ ns_out,
                                             uint32_t* __restrict__ err) {
  __shared__ uint32_t h[MAXA];
  __shared__ uint32_t bad;
  const uint32_t b = blockIdx.x;
  for (int i = threadIdx.x; i < MAXA; i += NT) h[i] = 0;
  if (threadIdx.x == 0) bad = 0;
  uint32_t nu = 0;
  for (int j = 0; j < 8; j++) nu += __popc(inuse[b * 8 + j]);
  const uint32_t alpha = nu + 2;
  const uint64_t o = sym_off[b];
  const uint64_t cap = sym_off[b + 1] - sym_off[b];
  const uint32_t n_in = nsyms[b];
  const uint32_t ns = (uint32_t)min((uint64_t)n_in, cap);
  __syncthreads();
  const uint16_t* S = syms + o;
  for (uint32_t i = threadIdx.x; i < ns; i += NT) {
    const uint32_t v = S[i];
    if (v < alpha) atomicAdd(&h[v], 1u);
    else bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ns_out[b] = ns;
    if (bad || n_in > cap) atomicOr(err, ERR_SYMBOL);
  }
  for (int i = threadIdx.x; i < MAXA; i += NT) freq[(size_t)b * MAXA + i] = h[i];
}

size_t block_tables_bytes() { return sizeof(BlockTables); }

// Scratch for huff_run: packed costs and per-table counts.
size_t huff_workspace_bytes(uint32_t nb) {
  return ((size_t)nb * MAXA * 8 + 255) / 256 * 256 + ((size_t)nb * MAXG * MAXA * 4 + 255) / 256 * 256 + 512;
}

// The Huffman stage of nb blocks (some possibly empty): counts (when
// a.count_freq: symbols given by the caller, validated), four passes of
// table assignment and build (with precomputed tables: one assignment),
// the final data bits, codes and selectors.
hipError_t huff_run(const HuffArgs& a, hipStream_t st) {
  if (!a.nb) return hipSuccess;
  BlockTables* tabs = (BlockTables*)a.tabs;
  uint64_t* cost = (uint64_t*)a.ws;
  uint32_t* tf = (uint32_t*)((char*)a.ws + ((size_t)a.nb * MAXA * 8 + 255) / 256 * 256);
  const uint32_t* nsyms = a.nsyms;
  if (a.count_freq) {
    hipLaunchKernelGGL(k_freq, dim3(a.nb), dim3(NT), 0, st, a.syms, a.sym_off, a.nsyms, a.inuse, a.freq, a.ns_eff,
                       a.err);
    nsyms = a.ns_eff;
  }
  const uint32_t g = persist_grid(a.tiles_cap, ONE_TILE_EACH);
  const int clamp = a.count_freq ? 1 : 0;
  // symbol counts are known on the device only: no algorithmic bytes recorded
  if (a.fixed) {
    ProfScope ps("huff_setup", st, 0.0);
    hipLaunchKernelGGL(k_huff_fixed_setup, dim3(a.nb), dim3(NT), 0, st, nsyms, a.inuse, tabs, tf, a.sel_base, a.gbits,
                       a.fixed, a.fixed_g);
  } else {
    ProfScope ps("huff_setup", st, 0.0);
    hipLaunchKernelGGL(k_huff_setup, dim3(a.nb), dim3(NT), 0, st, nsyms, a.freq, a.inuse, tabs, cost, tf, a.sel_base,
                       a.gbits);
  }
  // precomputed tables: one selector pass and no rebuild
  const int passes = a.fixed ? 1 : 4;
  for (int it = 0; it < passes; it++) {
    {
      ProfScope ps("huff_assign", st, 0.0);
      hipLaunchKernelGGL(k_huff_assign, dim3(g), dim3(NT), 0, st, 0, a.tile_blk, a.blk_tile0, a.syms, a.sym_base,
                         nsyms, a.sel_base, a.sel, (const uint64_t*)cost, tf, a.gbits, tabs, a.tile_groups, a.n_tiles,
                         a.tiles_cap, clamp);
    }
    if (a.fixed) break;
    ProfScope ps("huff_build", st, 0.0);
    hipLaunchKernelGGL(k_huff_build, dim3(a.nb, MAXG), dim3(BUILD_NT), 0, st, tabs, tf);
  }
  {
    ProfScope ps("huff_assign", st, 0.0);
    hipLaunchKernelGGL(k_huff_assign, dim3(g), dim3(NT), 0, st, 1, a.tile_blk, a.blk_tile0, a.syms, a.sym_base, nsyms,
                       a.sel_base, a.sel, (const uint64_t*)cost, tf, a.gbits, tabs, a.tile_groups, a.n_tiles,
                       a.tiles_cap, clamp);
  }
  ProfScope ps("huff_finish", st, 0.0);
  hipLaunchKernelGGL(k_huff_finish, dim3(a.nb), dim3(NT), 0, st, a.inuse, a.sel_base, (const uint8_t*)a.sel, a.selmtf,
                     tabs);
  return hipGetLastError();
}

// Groups per assign tile for a call with ng groups in all: smaller tiles
// when the large ones would leave most of the GPU idle.
uint32_t huff_assign_groups(uint64_t ng) {
  if (g_tune && (g_tune->assign_groups == ASSIGN_GROUPS || g_tune->assign_groups == ASSIGN_GROUPS_SMALL))
    return g_tune->assign_groups;
  return ng >= 1024ull * ASSIGN_GROUPS ? ASSIGN_GROUPS : ASSIGN_GROUPS_SMALL;
}

}  // namespace bzg
