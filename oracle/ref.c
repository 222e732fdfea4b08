/*
 * Tier-1 oracle: the bzip2 compression stages in plain C, for full-size
 * blocks.  TEST INFRASTRUCTURE ONLY: the product library never includes,
 * links or calls this file; only the tests, the smoke check and the CPU
 * baseline of the benchmark load it (through ctypes).  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * It computes exactly what the Python tier-0 oracle computes, with the same
 * plain algorithms:
 *   - block CRC bit by bit (bzip2 container; not in the paper);
 *   - RLE1 run by run (Sec. 3.2 run-length coding, bzip2's variant);
 *   - BWT as a comparison sort of the rotations (Sec. 3.1): qsort with
 *     memcmp on the doubled block, equal rotations by descending start index;
 *     a cyclically periodic block is sorted through its primitive root;
 *   - MTF with an explicit list over the in-use bytes (Sec. 3.3);
 *   - RUNA/RUNB zero runs, textbook Huffman by repeated selection of the two
 *     lightest nodes, the project's table heuristic (Sec. 3.4, Sec. 4);
 *   - an MSB-first bit writer; codes laid end to end (Figure 3).
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ CRC */

uint32_t ref_crc32(const uint8_t *p, uint64_t n) {
  uint32_t reg = 0xFFFFFFFFu;
  for (uint64_t i = 0; i < n; i++) {
    for (int bit = 7; bit >= 0; bit--) {
      uint32_t inbit = (p[i] >> bit) & 1u;
      uint32_t top = reg >> 31;
      reg <<= 1;
      if (top ^ inbit) reg ^= 0x04C11DB7u;
    }
  }
  return reg ^ 0xFFFFFFFFu;
}

/* ----------------------------------------------------------------- RLE1 */

/* out must hold 5 * ceil(n / 4) bytes; returns the encoded length. */
uint64_t ref_rle1(const uint8_t *in, uint64_t n, uint8_t *out) {
  uint64_t i = 0, o = 0;
  while (i < n) {
    uint8_t b = in[i];
    uint64_t r = 1;
    while (i + r < n && in[i + r] == b) r++;
    i += r;
    while (r > 0) {
      uint64_t c = r < 255 ? r : 255;
      if (c >= 4) {
        out[o++] = b; out[o++] = b; out[o++] = b; out[o++] = b;
        out[o++] = (uint8_t)(c - 4);
      } else {
        for (uint64_t k = 0; k < c; k++) out[o++] = b;
      }
      r -= c;
    }
  }
  return o;
}

/* RLE1 output length without writing it. */
uint64_t ref_rle1_len(const uint8_t *in, uint64_t n) {
  uint64_t i = 0, o = 0;
  while (i < n) {
    uint64_t r = 1;
    while (i + r < n && in[i + r] == in[i]) r++;
    i += r;
    o += 5 * (r / 255);
    r %= 255;
    o += r >= 4 ? 5 : r;
  }
  return o;
}

/* Cut every block whose RLE1 output exceeds `limit` after the longest input
 * prefix whose own RLE1 output fits (bisection: the prefix length is
 * monotone); the rest becomes the next block.  Empty blocks are dropped.
 * out_offs needs room for max_out + 1 entries; returns the new block count or
 * -1 when max_out is too small. */
int64_t ref_split_blocks(const uint8_t *in, const uint64_t *offs, uint32_t nb, uint64_t limit,
                         uint64_t *out_offs, uint64_t max_out) {
  uint64_t m = 0;
  out_offs[0] = offs[0];
  for (uint32_t k = 0; k < nb; k++) {
    uint64_t lo_off = offs[k], hi_off = offs[k + 1];
    while (hi_off > lo_off) {
      const uint8_t *raw = in + lo_off;
      uint64_t n = hi_off - lo_off, cut;
      if (ref_rle1_len(raw, n) <= limit) cut = n;
      else {
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
          uint64_t mid = (lo + hi + 1) / 2;
          if (ref_rle1_len(raw, mid) <= limit) lo = mid; else hi = mid - 1;
        }
        cut = lo;
      }
      if (m >= max_out) return -1;
      lo_off += cut;
      out_offs[++m] = lo_off;
    }
  }
  return (int64_t)m;
}

/* ------------------------------------------------------------------ BWT */

typedef struct { const uint8_t *ss; uint32_t len; } rot_ctx;

static int rot_cmp(const void *a, const void *b, void *arg) {
  const rot_ctx *c = (const rot_ctx *)arg;
  uint32_t i = *(const uint32_t *)a, j = *(const uint32_t *)b;
  int r = memcmp(c->ss + i, c->ss + j, c->len);
  if (r) return r;
  return (i > j) ? -1 : (i < j ? 1 : 0); /* equal: larger start first */
}

/* Smallest p dividing n with s cyclically p-periodic (n if none), from the
 * failure function of the string. */
uint32_t ref_cyclic_period(const uint8_t *s, uint32_t n) {
  if (n <= 1) return n;
  uint32_t *f = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
  f[0] = 0; f[1] = 0;
  uint32_t k = 0;
  for (uint32_t i = 1; i < n; i++) {
    while (k > 0 && s[i] != s[k]) k = f[k];
    if (s[i] == s[k]) k++;
    f[i + 1] = k;
  }
  uint32_t p = n - f[n];
  free(f);
  return (n % p == 0) ? p : n;
}

/* sa[n], last[n]; returns origPtr, or -1 on bad input / allocation failure. */
int64_t ref_bwt(const uint8_t *s, uint32_t n, uint32_t *sa, uint8_t *last) {
  if (n == 0) return -1;
  uint32_t p = ref_cyclic_period(s, n);
  uint8_t *ss = (uint8_t *)malloc(2 * (size_t)p);
  uint32_t *root = (uint32_t *)malloc(sizeof(uint32_t) * p);
  if (!ss || !root) { free(ss); free(root); return -1; }
  memcpy(ss, s, p);
  memcpy(ss + p, s, p);
  for (uint32_t i = 0; i < p; i++) root[i] = i;
  rot_ctx ctx = {ss, p};
  qsort_r(root, p, sizeof(uint32_t), rot_cmp, &ctx);
  uint32_t copies = n / p, k = 0;
  int64_t optr = -1;
  for (uint32_t r = 0; r < p; r++) {
    for (uint32_t c = copies; c-- > 0;) { /* equal rotations, descending */
      uint32_t i = root[r] + c * p;
      sa[k] = i;
      last[k] = s[(i + n - 1) % n];
      if (i == 0) optr = k;
      k++;
    }
  }
  free(ss);
  free(root);
  return optr;
}

/* Property check of a suffix order: sa is a permutation of 0..n-1 and every
 * adjacent pair is in order (rotations compared as unsigned bytes, equal ones
 * larger start first).  Returns -1 if it holds, else the first bad row (or n
 * for a non-permutation). */
int64_t ref_check_sa(const uint8_t *s, uint32_t n, const uint32_t *sa) {
  uint8_t *seen = (uint8_t *)calloc(n ? n : 1, 1);
  for (uint32_t k = 0; k < n; k++) {
    if (sa[k] >= n || seen[sa[k]]) { free(seen); return n; }
    seen[sa[k]] = 1;
  }
  free(seen);
  uint32_t p = ref_cyclic_period(s, n);
  uint8_t *ss = (uint8_t *)malloc(2 * (size_t)n);
  memcpy(ss, s, n);
  memcpy(ss + n, s, n);
  rot_ctx ctx = {ss, p}; /* rotations agreeing on p bytes of a p-periodic block are equal */
  for (uint32_t k = 0; k + 1 < n; k++) {
    if (rot_cmp(&sa[k], &sa[k + 1], &ctx) >= 0) { free(ss); return k; }
  }
  free(ss);
  return -1;
}

/* ------------------------------------------------- MTF and RUNA / RUNB */

static uint32_t put_run(uint16_t *out, uint32_t o, uint64_t r) {
  while (r > 0) {
    if (r & 1) { out[o++] = 0; r = (r - 1) >> 1; }
    else       { out[o++] = 1; r = (r - 2) >> 1; }
  }
  return o;
}

/* out needs n + 1 slots.  used[256] receives 0/1 flags.  Returns the symbol
 * count (EOB included); *n_inuse gets the in-use count. */
uint32_t ref_mtf_zrle(const uint8_t *last, uint32_t n, uint16_t *out,
                      uint8_t *used, uint32_t *n_inuse, uint8_t *mtf /* nullable, n */) {
  uint8_t list[256];
  uint32_t nu = 0;
  memset(used, 0, 256);
  for (uint32_t i = 0; i < n; i++) used[last[i]] = 1;
  for (int b = 0; b < 256; b++) if (used[b]) list[nu++] = (uint8_t)b;
  uint32_t o = 0;
  uint64_t run = 0;
  for (uint32_t i = 0; i < n; i++) {
    uint32_t v = 0;
    while (list[v] != last[i]) v++;
    for (uint32_t j = v; j > 0; j--) list[j] = list[j - 1];
    list[0] = last[i];
    if (mtf) mtf[i] = (uint8_t)v;
    if (v == 0) { run++; continue; }
    o = put_run(out, o, run);
    run = 0;
    out[o++] = (uint16_t)(v + 1);
  }
  o = put_run(out, o, run);
  out[o++] = (uint16_t)(nu + 1);
  *n_inuse = nu;
  return o;
}

/* ------------------------------------------------------------- Huffman */

#define MAXA 258
#define MAXG 6
#define GRP 50
#define MAXLEN 17

/* Repeatedly merge the two lightest live nodes by (weight, id); leaves are
 * 0..a-1, internal nodes a, a+1, ... in creation order.  Lengths = depths.
 * While a length exceeds MAXLEN, w <- 1 + w/2 and rebuild. */
void ref_huffman_lengths(const uint32_t *freq, int a, uint8_t *len) {
  uint64_t w[2 * MAXA];
  int parent[2 * MAXA], live[2 * MAXA];
  for (int i = 0; i < a; i++) w[i] = freq[i] ? freq[i] : 1;
  for (;;) {
    int nodes = a;
    for (int i = 0; i < 2 * a; i++) { parent[i] = -1; live[i] = i < a; }
    for (int step = 0; step < a - 1; step++) {
      int x = -1, y = -1;
      for (int i = 0; i < nodes; i++) {
        if (!live[i]) continue;
        if (x < 0 || w[i] < w[x]) { y = x; x = i; }
        else if (y < 0 || w[i] < w[y]) y = i;
      }
      /* ties: ids are scanned ascending and only a strictly smaller weight
       * displaces, so (weight, id) order is kept */
      w[nodes] = w[x] + w[y];
      parent[x] = nodes; parent[y] = nodes;
      live[x] = 0; live[y] = 0; live[nodes] = 1;
      nodes++;
    }
    int maxd = 0;
    for (int i = 0; i < a; i++) {
      int d = 0, v = i;
      while (parent[v] >= 0) { v = parent[v]; d++; }
      len[i] = (uint8_t)d;
      if (d > maxd) maxd = d;
    }
    if (maxd <= MAXLEN) return;
    for (int i = 0; i < a; i++) w[i] = 1 + w[i] / 2;
  }
}

void ref_canonical_codes(const uint8_t *len, int a, uint32_t *code) {
  int mn = 32, mx = 0;
  for (int i = 0; i < a; i++) { if (len[i] < mn) mn = len[i]; if (len[i] > mx) mx = len[i]; }
  uint32_t c = 0;
  for (int l = mn; l <= mx; l++) {
    for (int i = 0; i < a; i++) if (len[i] == l) code[i] = c++;
    c <<= 1;
  }
}

int ref_n_tables(uint32_t nsyms, int a) {
  int g = nsyms < 200 ? 2 : nsyms < 600 ? 3 : nsyms < 1200 ? 4 : nsyms < 2400 ? 5 : 6;
  return g < a ? g : a;
}

/* lens[MAXG*MAXA], sel[ceil(nsyms/50)].  Returns the table count. */
int ref_tables(const uint16_t *syms, uint32_t nsyms, int a, uint8_t *lens, uint8_t *sel) {
  uint32_t freq[MAXA] = {0};
  for (uint32_t i = 0; i < nsyms; i++) freq[syms[i]]++;
  int g = ref_n_tables(nsyms, a);
  uint32_t nsel = (nsyms + GRP - 1) / GRP;
  /* initial equal-frequency partition */
  uint64_t rem = nsyms;
  int gs = 0;
  for (int t = 0; t < g; t++) {
    int left = g - t, ge;
    if (left == 1) ge = a - 1;
    else {
      ge = gs;
      uint64_t acc = freq[gs];
      while (ge + 1 <= a - left && acc * (uint64_t)left < rem) { ge++; acc += freq[ge]; }
    }
    uint64_t part = 0;
    for (int v = 0; v < a; v++) {
      lens[t * MAXA + v] = (v >= gs && v <= ge) ? 0 : 15;
      if (v >= gs && v <= ge) part += freq[v];
    }
    rem -= part;
    gs = ge + 1;
  }
  uint32_t tf[MAXG][MAXA];
  for (int it = 0; it < 4; it++) {
    memset(tf, 0, sizeof(tf));
    for (uint32_t j = 0; j < nsel; j++) {
      uint32_t lo = j * GRP, hi = lo + GRP < nsyms ? lo + GRP : nsyms;
      uint32_t best = 0, bestc = 0xFFFFFFFFu;
      for (int t = 0; t < g; t++) {
        uint32_t c = 0;
        for (uint32_t i = lo; i < hi; i++) c += lens[t * MAXA + syms[i]];
        if (c < bestc) { bestc = c; best = (uint32_t)t; }
      }
      sel[j] = (uint8_t)best;
      for (uint32_t i = lo; i < hi; i++) tf[best][syms[i]]++;
    }
    for (int t = 0; t < g; t++) ref_huffman_lengths(tf[t], a, lens + t * MAXA);
  }
  return g;
}

/* ---------------------------------------------------------- bit writer */

typedef struct { uint8_t *buf; uint64_t cap, bits; } bw_t;

static void bw_put(bw_t *w, uint64_t v, int n) {
  for (int k = n - 1; k >= 0; k--) {
    if ((w->bits >> 3) >= w->cap) {
      uint64_t nc = w->cap ? 2 * w->cap : 4096;
      w->buf = (uint8_t *)realloc(w->buf, nc);
      memset(w->buf + w->cap, 0, nc - w->cap);
      w->cap = nc;
    }
    if ((v >> k) & 1) w->buf[w->bits >> 3] |= (uint8_t)(0x80u >> (w->bits & 7));
    w->bits++;
  }
}

/* Symbol map, G, nSel, MTF'd unary selectors, delta-coded lengths, codes. */
static void write_body(bw_t *w, const uint8_t *used, int g, uint32_t nsel, const uint8_t *sel,
                       const uint8_t *lens, int a, const uint16_t *syms, uint32_t nsyms) {
  int ranges[16];
  for (int i = 0; i < 16; i++) {
    ranges[i] = 0;
    for (int j = 0; j < 16; j++) ranges[i] |= used[16 * i + j];
    bw_put(w, (uint64_t)ranges[i], 1);
  }
  for (int i = 0; i < 16; i++)
    if (ranges[i])
      for (int j = 0; j < 16; j++) bw_put(w, used[16 * i + j], 1);
  bw_put(w, (uint64_t)g, 3);
  bw_put(w, nsel, 15);
  uint8_t stack[MAXG];
  for (int t = 0; t < g; t++) stack[t] = (uint8_t)t;
  for (uint32_t j = 0; j < nsel; j++) {
    int v = 0;
    while (stack[v] != sel[j]) v++;
    for (int k = v; k > 0; k--) stack[k] = stack[k - 1];
    stack[0] = sel[j];
    for (int k = 0; k < v; k++) bw_put(w, 1, 1);
    bw_put(w, 0, 1);
  }
  for (int t = 0; t < g; t++) {
    int cur = lens[t * MAXA];
    bw_put(w, (uint64_t)cur, 5);
    for (int i = 0; i < a; i++) {
      int l = lens[t * MAXA + i];
      while (cur < l) { bw_put(w, 2, 2); cur++; }
      while (cur > l) { bw_put(w, 3, 2); cur--; }
      bw_put(w, 0, 1);
    }
  }
  uint32_t codes[MAXG][MAXA];
  for (int t = 0; t < g; t++) ref_canonical_codes(lens + t * MAXA, a, codes[t]);
  for (uint32_t i = 0; i < nsyms; i++) {
    int t = sel[i / GRP];
    bw_put(w, codes[t][syms[i]], lens[t * MAXA + syms[i]]);
  }
}

/* ------------------------------------------------------------- blocks */

typedef struct {
  uint32_t crc, orig_ptr, n_rle1;
  bw_t body; /* bits after origPtr */
  int err;
} block_out;

/* Precomputed tables (Sec. 4): lens over the 258 symbols of a block with
 * every byte in use, g of them.  A block of alphabet a uses symbols
 * 0..a-2 as they are and takes symbol 257's length for its EOB; each group
 * picks the cheapest table (lowest index on ties).  No table is built. */
static int fixed_tables(const uint8_t *fixed, int fg, const uint16_t *syms, uint32_t nsyms, int a,
                        uint8_t *lens, uint8_t *sel) {
  for (int t = 0; t < fg; t++)
    for (int v = 0; v < a; v++) lens[t * MAXA + v] = fixed[t * MAXA + (v == a - 1 ? MAXA - 1 : v)];
  uint32_t nsel = (nsyms + GRP - 1) / GRP;
  for (uint32_t j = 0; j < nsel; j++) {
    uint32_t lo = j * GRP, hi = lo + GRP < nsyms ? lo + GRP : nsyms;
    uint32_t best = 0, bestc = 0xFFFFFFFFu;
    for (int t = 0; t < fg; t++) {
      uint32_t c = 0;
      for (uint32_t i = lo; i < hi; i++) c += lens[t * MAXA + syms[i]];
      if (c < bestc) { bestc = c; best = (uint32_t)t; }
    }
    sel[j] = (uint8_t)best;
  }
  return fg;
}

static const uint8_t *g_fixed;  /* set for the duration of ref_compress_fixed */
static int g_fixed_g;

static void encode_one(const uint8_t *raw, uint64_t n, block_out *bo) {
  memset(bo, 0, sizeof(*bo));
  bo->crc = ref_crc32(raw, n);
  uint8_t *r1 = (uint8_t *)malloc(5 * ((n + 3) / 4) + 1);
  uint64_t m = ref_rle1(raw, n, r1);
  bo->n_rle1 = (uint32_t)m;
  uint32_t *sa = (uint32_t *)malloc(sizeof(uint32_t) * m);
  uint8_t *last = (uint8_t *)malloc(m);
  uint16_t *syms = (uint16_t *)malloc(sizeof(uint16_t) * (m + 1));
  int64_t optr = ref_bwt(r1, (uint32_t)m, sa, last);
  if (optr < 0) { bo->err = 1; goto done; }
  bo->orig_ptr = (uint32_t)optr;
  uint8_t used[256];
  uint32_t nu;
  uint32_t ns = ref_mtf_zrle(last, (uint32_t)m, syms, used, &nu, NULL);
  int a = (int)nu + 2;
  uint8_t lens[MAXG * MAXA];
  uint32_t nsel = (ns + GRP - 1) / GRP;
  uint8_t *sel = (uint8_t *)malloc(nsel);
  int g = g_fixed ? fixed_tables(g_fixed, g_fixed_g, syms, ns, a, lens, sel) : ref_tables(syms, ns, a, lens, sel);
  write_body(&bo->body, used, g, nsel, sel, lens, a, syms, ns);
  free(sel);
done:
  free(r1); free(sa); free(last); free(syms);
}

typedef struct {
  const uint8_t *in;
  const uint64_t *offs;
  uint32_t nb;
  block_out *bo;
  volatile uint32_t next;
  pthread_mutex_t mu;
} pool_t;

static void *worker(void *arg) {
  pool_t *P = (pool_t *)arg;
  for (;;) {
    pthread_mutex_lock(&P->mu);
    uint32_t k = P->next++;
    pthread_mutex_unlock(&P->mu);
    if (k >= P->nb) return NULL;
    encode_one(P->in + P->offs[k], P->offs[k + 1] - P->offs[k], &P->bo[k]);
  }
}

/* Compress blocks [offs[k], offs[k+1]) into one stream with header digit
 * `level`; blocks are first cut so that no RLE1 output exceeds 100000*level.
 * Returns the stream length, 0 when out_cap is too small (then *need receives
 * the length) or -1 on error. */
int64_t ref_compress(const uint8_t *in, const uint64_t *offs0, uint32_t nb0, int level,
                     uint8_t *out, uint64_t out_cap, uint64_t *need, int threads) {
  uint64_t total = nb0 ? offs0[nb0] - offs0[0] : 0;
  uint64_t max_out = nb0 + total / 50000 + 2;
  uint64_t *offs = (uint64_t *)malloc(sizeof(uint64_t) * (max_out + 1));
  int64_t nbs = nb0 ? ref_split_blocks(in, offs0, nb0, 100000ull * (uint64_t)level, offs, max_out) : 0;
  if (nbs < 0) { free(offs); return -1; }
  uint32_t nb = (uint32_t)nbs;
  block_out *bo = (block_out *)calloc(nb ? nb : 1, sizeof(block_out));
  pool_t P = {in, offs, nb, bo, 0, PTHREAD_MUTEX_INITIALIZER};
  if (threads < 1) threads = 1;
  pthread_t th[256];
  if (threads > 256) threads = 256;
  for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, worker, &P);
  for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
  for (uint32_t k = 0; k < nb; k++) {
    if (bo[k].err) { free(bo); free(offs); return -1; }
  }
  bw_t w = {0, 0, 0};
  bw_put(&w, 'B', 8); bw_put(&w, 'Z', 8); bw_put(&w, 'h', 8); bw_put(&w, (uint64_t)('0' + level), 8);
  uint32_t comb = 0;
  for (uint32_t k = 0; k < nb; k++) {
    bw_put(&w, 0x314159265359ull, 48);
    bw_put(&w, bo[k].crc, 32);
    bw_put(&w, 0, 1);
    bw_put(&w, bo[k].orig_ptr, 24);
    for (uint64_t b = 0; b < bo[k].body.bits; b++)
      bw_put(&w, (bo[k].body.buf[b >> 3] >> (7 - (b & 7))) & 1, 1);
    comb = ((comb << 1) | (comb >> 31)) ^ bo[k].crc;
    free(bo[k].body.buf);
  }
  bw_put(&w, 0x177245385090ull, 48);
  bw_put(&w, comb, 32);
  free(bo);
  free(offs);
  uint64_t len = (w.bits + 7) / 8;
  if (need) *need = len;
  if (len > out_cap) { free(w.buf); return 0; }
  memcpy(out, w.buf, len);
  free(w.buf);
  return (int64_t)len;
}

/* ref_compress with precomputed tables (fixed: g x 258 lengths, row
 * stride 258).  Not reentrant (the tables are held in a file-scope pointer
 * for the workers). */
int64_t ref_compress_fixed(const uint8_t *in, const uint64_t *offs0, uint32_t nb0, int level,
                           const uint8_t *fixed, int g, uint8_t *out, uint64_t out_cap, uint64_t *need,
                           int threads) {
  g_fixed = fixed;
  g_fixed_g = g;
  int64_t r = ref_compress(in, offs0, nb0, level, out, out_cap, need, threads);
  g_fixed = NULL;
  g_fixed_g = 0;
  return r;
}

/* Stage entry for tests: the body bits (symbol map .. last code) of one
 * block given its MTF/RUNA-RUNB symbols.  Returns the bit count, or -1 when
 * cap_bytes is too small.  lens_out (MAXG*MAXA), sel_out and g_out may be
 * NULL. */
int64_t ref_body(const uint16_t *syms, uint32_t nsyms, const uint8_t *used,
                 uint8_t *out, uint64_t cap_bytes, uint8_t *lens_out, uint8_t *sel_out,
                 int *g_out) {
  int nu = 0;
  for (int b = 0; b < 256; b++) nu += used[b] ? 1 : 0;
  int a = nu + 2;
  uint8_t lens[MAXG * MAXA];
  uint32_t nsel = (nsyms + GRP - 1) / GRP;
  uint8_t *sel = (uint8_t *)malloc(nsel ? nsel : 1);
  int g = ref_tables(syms, nsyms, a, lens, sel);
  bw_t w = {0, 0, 0};
  write_body(&w, used, g, nsel, sel, lens, a, syms, nsyms);
  if (lens_out) memcpy(lens_out, lens, sizeof(lens));
  if (sel_out) memcpy(sel_out, sel, nsel);
  if (g_out) *g_out = g;
  free(sel);
  int64_t bits = (int64_t)w.bits;
  if ((w.bits + 7) / 8 > cap_bytes) { free(w.buf); return -1; }
  memset(out, 0, (w.bits + 7) / 8);
  if (w.bits) memcpy(out, w.buf, (w.bits + 7) / 8);
  free(w.buf);
  return bits;
}
