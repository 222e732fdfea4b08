// C ABI: argument checking, workspace planning from host bounds, and the
// launch sequence of every entry point declared in include/bzgpu.h.  No call
// reads anything back from the device: data-dependent sizes are planned by
// the kernels in plan.hip, and kernel-side errors go to the context's status
// word, reported by bzg_check.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/bzgpu.h"
#include "internal.hpp"
#include "plan.hpp"

namespace bzg {
// launchers from the kernel translation units
hipError_t rle1_tiles(const uint8_t*, uint32_t, const uint32_t*, const uint32_t*, const uint32_t*, const uint64_t*,
                      const uint32_t*, const uint32_t*, void*, hipStream_t);
hipError_t rle1_blocks(uint32_t, const uint32_t*, const uint64_t*, const uint32_t*, const void*, uint32_t*, uint32_t*,
                       uint32_t*, uint32_t*, hipStream_t);
hipError_t rle1_emit(const uint8_t*, uint32_t, const uint32_t*, const uint32_t*, const uint32_t*, const uint64_t*,
                     const uint32_t*, const uint32_t*, const uint32_t*, uint8_t*, hipStream_t);
hipError_t rle1_split(const uint8_t*, const uint64_t*, uint32_t, const uint32_t*, const void*, const uint32_t*,
                      const uint32_t*, const uint32_t*, const uint32_t*, uint32_t, uint32_t, uint64_t*, uint32_t*,
                      hipStream_t);
size_t rle_tile_bytes();
uint32_t mtf_chunk_rows(uint64_t rows, uint32_t nb);
size_t mtf_workspace_bytes(uint64_t rows, uint32_t nb);
hipError_t mtf_run(const uint8_t*, const uint32_t*, uint32_t, uint64_t, const uint32_t*, const uint32_t*,
                   const uint32_t*, void*, size_t, uint16_t*, const uint64_t*, uint32_t*, uint32_t*, uint32_t*, uint32_t*,
                   std::string&, hipStream_t);
size_t huff_workspace_bytes(uint32_t nb);
uint32_t huff_assign_groups(uint64_t ng);
hipError_t huff_run(const HuffArgs&, hipStream_t);
hipError_t pack_layout(uint32_t, uint32_t, const uint32_t*, const uint64_t*, const void*, int, const uint64_t*,
                       uint64_t*, const uint32_t*, uint64_t*, uint64_t*, uint32_t*, const uint32_t*, uint32_t*,
                       uint32_t*, hipStream_t);
hipError_t zero_streams(uint32_t, uint64_t, const uint64_t*, const uint64_t*, uint32_t*, const uint32_t*, hipStream_t);
hipError_t zero_range(uint32_t*, uint64_t, const uint32_t*, hipStream_t);
hipError_t pack_run(uint32_t, const void*, int, const uint64_t*, const uint32_t*, const uint32_t*, const uint32_t*,
                    const uint64_t*, const uint8_t*, const uint8_t*, const uint64_t*, const uint32_t*, uint32_t,
                    const uint32_t*, const uint32_t*, const uint16_t*, const uint64_t*, const uint32_t*, int, uint32_t,
                    const uint64_t*, const uint64_t*, uint32_t*, const uint32_t*, hipStream_t);
hipError_t tables_export(uint32_t, const void*, uint8_t*, hipStream_t);
}  // namespace bzg

namespace bzg {

thread_local Profiler* g_prof = nullptr;
thread_local const Tune* g_tune = nullptr;

ProfScope::ProfScope(const char* name, hipStream_t s, double bytes, const uint32_t* count0, double per0,
                     const uint32_t* count1, double per1)
    : st(s), c0(count0), c1(count1) {
  if (g_prof && g_prof->on) {
    Profiler::Pending p{name, nullptr, nullptr, bytes, {per0, per1}, -1};
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    (void)hipEventRecord(p.a, s);
    if ((c0 || c1) && g_prof->slots && g_prof->used + 2 <= g_prof->nslots) {
      p.slot = g_prof->used;
      g_prof->used += 2;
    }
    g_prof->pending.push_back(p);
    live = true;
  }
}

ProfScope::~ProfScope() {
  if (!live) return;
  Profiler::Pending& p = g_prof->pending.back();
  (void)hipEventRecord(p.b, st);
  // the counts as they are right after the launch (the records are reused
  // later in the call)
  if (p.slot >= 0) {
    if (c0) (void)hipMemcpyAsync(g_prof->slots + p.slot, c0, 4, hipMemcpyDeviceToDevice, st);
    if (c1) (void)hipMemcpyAsync(g_prof->slots + p.slot + 1, c1, 4, hipMemcpyDeviceToDevice, st);
  }
}

void Profiler::collect() {
  std::vector<uint32_t> h(used);
  if (used) {
    (void)hipDeviceSynchronize();
    (void)hipMemcpy(h.data(), slots, (size_t)used * 4, hipMemcpyDeviceToHost);
  }
  for (auto& p : pending) {
    float ms = 0;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ProfRec& r = acc[p.name];
      r.ms += ms;
      double b = p.bytes;
      if (p.slot >= 0) b += p.per[0] * h[p.slot] + p.per[1] * h[p.slot + 1];
      r.bytes += b;
      r.launches++;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  pending.clear();
  used = 0;
}

}  // namespace bzg

using namespace bzg;

// Scratch of compress_blocks_noalloc: a file-scope device array, one per
// GPU, allocated when the code object loads and held until the process
// ends.  Host code uses the per-device address from hipGetSymbolAddress
// (bzg_ctx::scratch), never this name.
constexpr size_t SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

struct bzg_ctx {
  std::mutex mu;  // calls on one context enqueue one at a time
  int device = 0;
  Profiler prof;
  std::string err;
  uint32_t* status = nullptr;  // device: kernel-side error flags
  // device: 4 x 256 byte-step tables (slicing by 4), 64 powers x^(8*2^j),
  // 256 tile shifts (mod P)
  uint32_t* crc_tab = nullptr;
  // workspace pool for calls without d_ws (stream-ordered growth)
  void* pool = nullptr;
  size_t pool_cap = 0;
  hipEvent_t pool_ev = nullptr;  // the end of the last call that used the pool
  bool pool_used = false;
  // pinned arena for uploads of host tables: two halves, each with the event
  // that follows its last copies
  char* stage = nullptr;
  size_t stage_half = 0;
  hipEvent_t stage_ev[2] = {nullptr, nullptr};
  bool stage_used[2] = {false, false};
  int stage_next = 0;
  void* scratch = nullptr;  // this device's copy of `scratch`
  // launch parameters: set explicitly (bzg_set_tune), or per size bucket
  // from bzg_tune and the tune cache file
  Tune tune;
  bool tune_set = false;
  std::map<uint32_t, Tune> tune_table;
  std::string tune_path, tune_id;
  // precomputed Huffman tables (bzg_set_fixed_tables): MAXG x MAXA lengths
  uint8_t* fixed_tab = nullptr;
  int fixed_g = 0;
  // compress_host: two input and two output buffers on the device, two
  // pinned input halves (for pageable inputs), pinned size words, the copy
  // streams and their events; kept between calls, grown on demand
  struct HostIo {
    size_t in_cap = 0, out_cap = 0, pin_cap = 0;
    uint8_t *din[2] = {nullptr, nullptr}, *dout[2] = {nullptr, nullptr}, *pin[2] = {nullptr, nullptr};
    uint64_t* dsize = nullptr;  // device: stream sizes of the two buffers
    uint64_t* hsize = nullptr;  // pinned: their copies
    hipStream_t up = nullptr, down = nullptr;
    hipEvent_t in_ev[2] = {nullptr, nullptr}, comp_ev[2] = {nullptr, nullptr}, out_ev[2] = {nullptr, nullptr};
  } hio;
  // decompress: the streams the longer blocks are decoded on, and the
  // events that fork them from the call's stream and join them back
  hipStream_t dec_side[2] = {nullptr, nullptr};
  hipEvent_t dec_fork = nullptr, dec_join[2] = {nullptr, nullptr};
};

namespace {

int fail(bzg_ctx* c, int code, const std::string& m) {
  c->err = m;
  return code;
}

int hip_fail(bzg_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return BZG_EHIP;
}

#define HIPX(call)                                         \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// CRC helper tables (built on the host from the polynomial).  tab[k*256 + b]
// is the register after k + 1 byte steps from b << 24 with zero input: the
// slicing-by-4 tables (Kounavis and Berry), k = 0 being the one-byte table.
void crc_tables(uint32_t* tab, uint32_t* pw) {
  const uint32_t P = 0x04C11DB7u;
  for (uint32_t b = 0; b < 256; b++) {
    uint32_t r = b << 24;
    for (int i = 0; i < 8; i++) r = (r & 0x80000000u) ? (r << 1) ^ P : (r << 1);
    tab[b] = r;
  }
  for (int k = 1; k < 4; k++)
    for (uint32_t b = 0; b < 256; b++) {
      const uint32_t r = tab[(k - 1) * 256 + b];
      tab[k * 256 + b] = (r << 8) ^ tab[r >> 24];
    }
  auto mul = [&](uint32_t a, uint32_t c) {
    uint32_t r = 0;
    for (int i = 31; i >= 0; i--) {
      r = (r << 1) ^ ((r & 0x80000000u) ? P : 0u);
      if ((c >> i) & 1u) r ^= a;
    }
    return r;
  };
  uint32_t x8 = 0x100u;  // x^8
  pw[0] = x8;
  for (int j = 1; j < 64; j++) pw[j] = mul(pw[j - 1], pw[j - 1]);
  // pw[64 + t] = x^(8 * 16 * (255 - t)): shift of thread t's 16 bytes to the
  // end of a full 4096-byte tile
  uint32_t x128 = pw[4];  // x^(8*16)
  uint32_t acc = 1;
  for (int t = 255; t >= 0; t--) {
    pw[64 + t] = acc;
    acc = mul(acc, x128);
  }
}

// Carves a workspace into 256-byte aligned arrays.  With base == nullptr it
// only adds up the size (the same sequence of takes sizes and carves).
struct Carve {
  char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t n) {
    size_t a = (used + 255) & ~size_t(255);
    used = a + n * sizeof(T);
    return base ? reinterpret_cast<T*>(base + a) : nullptr;
  }
};

bool offsets_ok(const uint64_t* h, uint32_t nb) {
  for (uint32_t k = 0; k < nb; k++)
    if (h[k + 1] < h[k]) return false;
  return true;
}

// Routes instrumented launches of one API call to the context's profiler.
struct ProfGuard {
  explicit ProfGuard(bzg_ctx* x) { g_prof = &x->prof; }
  ~ProfGuard() { g_prof = nullptr; }
};

// The launch parameters of a call over `total` bytes in `nb` blocks: the
// explicit ones, else the tuned entry of its size bucket, else the built-in
// choices (null).
uint32_t tune_bucket(uint64_t total, uint32_t nb) {
  uint32_t a = 0, b = 0;
  while (a < 63 && (2ull << a) <= total) a++;
  while (b < 31 && (2u << b) <= nb) b++;
  return (a << 8) | b;
}
const Tune* pick_tune(bzg_ctx* c, uint64_t total, uint32_t nb) {
  if (c->tune_set) return &c->tune;
  auto it = c->tune_table.find(tune_bucket(total, nb));
  return it == c->tune_table.end() ? nullptr : &it->second;
}
struct TuneGuard {
  TuneGuard(bzg_ctx* c, const uint64_t* h_off, uint32_t nb) {
    g_tune = pick_tune(c, nb && h_off ? h_off[nb] - h_off[0] : 0, nb);
  }
  ~TuneGuard() { g_tune = nullptr; }
};

// Workspace for a call: the caller's, or the context's pool (grown in
// stream order: the old pool is freed once `st` has passed every earlier
// call that used it).
int get_ws(bzg_ctx* ctx, void* d_ws, size_t ws_bytes, size_t need, hipStream_t st, void** out) {
  if (d_ws) {
    if (ws_bytes < need)
      return fail(ctx, BZG_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes; the call needs " +
                                           std::to_string(need));
    if ((uintptr_t)d_ws & 255) return fail(ctx, BZG_EINVAL, "d_ws must be 256-byte aligned");
    *out = d_ws;
    return 0;
  }
  if (ctx->pool_used) HIPX(hipStreamWaitEvent(st, ctx->pool_ev, 0));
  if (ctx->pool_cap < need) {
    if (ctx->pool) {
      HIPX(hipFreeAsync(ctx->pool, st));
      ctx->pool = nullptr;
      ctx->pool_cap = 0;
    }
    const size_t want = need + need / 8 + (1 << 20);
    if (hipMallocAsync(&ctx->pool, want, st) != hipSuccess) {
      (void)hipGetLastError();
      ctx->pool = nullptr;
      return fail(ctx, BZG_ENOMEM, "device workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->pool_cap = want;
  }
  *out = ctx->pool;
  return 0;
}

// Marks the end of a call's work on the pool (when it used the pool).
int end_ws(bzg_ctx* ctx, void* d_ws, hipStream_t st) {
  if (!d_ws) {
    HIPX(hipEventRecord(ctx->pool_ev, st));
    ctx->pool_used = true;
  }
  return 0;
}

// Host tables copied into the workspace through the pinned arena: the
// arena's halves alternate, and a half is refilled only after the copies
// last made from it have completed (normally long done).
struct Upload {
  void* dst;
  const void* src;
  size_t bytes;
};
int upload(bzg_ctx* ctx, std::initializer_list<Upload> ups, hipStream_t st) {
  size_t tot = 0;
  for (const Upload& u : ups) tot += (u.bytes + 255) & ~size_t(255);
  if (tot == 0) return 0;
  if (tot > ctx->stage_half) {  // grow: wait for both halves' copies first
    for (int h = 0; h < 2; h++)
      if (ctx->stage_used[h]) HIPX(hipEventSynchronize(ctx->stage_ev[h]));
    if (ctx->stage) HIPX(hipHostFree(ctx->stage));
    ctx->stage = nullptr;
    const size_t half = std::max(tot, ctx->stage_half * 2);
    if (hipHostMalloc((void**)&ctx->stage, 2 * half, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ctx->stage = nullptr;
      ctx->stage_half = 0;
      return fail(ctx, BZG_ENOMEM, "pinned host allocation failed");
    }
    ctx->stage_half = half;
    ctx->stage_used[0] = ctx->stage_used[1] = false;
  }
  const int h = ctx->stage_next;
  ctx->stage_next ^= 1;
  if (ctx->stage_used[h]) HIPX(hipEventSynchronize(ctx->stage_ev[h]));
  char* p = ctx->stage + (size_t)h * ctx->stage_half;
  size_t at = 0;
  for (const Upload& u : ups) {
    if (!u.bytes) continue;
    memcpy(p + at, u.src, u.bytes);
    HIPX(hipMemcpyAsync(u.dst, p + at, u.bytes, hipMemcpyHostToDevice, st));
    at += (u.bytes + 255) & ~size_t(255);
  }
  HIPX(hipEventRecord(ctx->stage_ev[h], st));
  ctx->stage_used[h] = true;
  return 0;
}

// ------------------------------------------------------------ compress plan

// Host bounds of a compress call, from the input offsets alone.
struct CBounds {
  uint32_t nb = 0, nslot = 0, L = 0;
  bool direct = true;  // every block is one slot (none empty, none that may need cutting)
  uint64_t total = 0;
  uint32_t in_tiles = 0, slot_tiles = 0, rows = 0, max_len = 0, sort_tiles = 0, mtf_ch = 0, chunks = 0;
  uint32_t groups = 0, atg = 0, asg_tiles = 0, pack_tiles = 0;
  uint64_t max_words = 0;  // largest stream, in 32-bit words
};

uint64_t compress_bound(uint64_t n_bytes, uint32_t n_blocks) {
  // every RLE1 byte becomes at most one 17-bit code (plus RUNA/RUNB digits,
  // which only replace zeros); generous per-block header allowance
  uint64_t rle = n_bytes + n_bytes / 4 + 4;
  uint64_t blocks = (uint64_t)n_blocks + rle / 100000 + 2;
  uint64_t bits = 32 + 80 + blocks * (105 + 16 + 256 + 18 + 6 * (5 + 258 * 33)) + rle * 17 + (rle / 50 + blocks) * 7;
  return ((bits + 7) / 8 + 3) & ~uint64_t(3);
}

CBounds compress_bounds(const uint64_t* h_off, uint32_t nb, int level, const uint32_t* h_rb, uint32_t n_req) {
  CBounds c;
  c.nb = nb;
  c.L = 100000u * (uint32_t)level;
  uint64_t rows = 0;
  for (uint32_t k = 0; k < nb; k++) {
    const uint64_t n = h_off[k + 1] - h_off[k];
    const uint32_t pm = max_pieces(n, c.L);
    c.nslot += pm;
    // slots are then the input blocks themselves; an empty block has no slot,
    // so it takes the planned path too
    if (pm != 1) c.direct = false;
    if (pm > 1) c.in_tiles += (uint32_t)((n + RLE_TILE - 1) / RLE_TILE);
    c.slot_tiles += (uint32_t)((n + RLE_TILE - 1) / RLE_TILE) + (pm ? pm - 1 : 0);
    const uint64_t r = std::min<uint64_t>(n + n / 4, (uint64_t)pm * c.L);
    rows += r;
    c.max_len = (uint32_t)std::max<uint64_t>(c.max_len, std::min<uint64_t>(n + n / 4, c.L));
  }
  c.total = nb ? h_off[nb] - h_off[0] : 0;
  c.rows = (uint32_t)std::min<uint64_t>(rows, 0xFFFFFFF0ull);
  c.sort_tiles = c.rows / RADIX_TILE + c.nslot + 1;
  c.mtf_ch = mtf_chunk_rows(c.rows, c.nslot);
  c.chunks = c.rows / c.mtf_ch + c.nslot + 1;
  c.groups = c.rows / GROUP + c.nslot + 1;
  c.atg = huff_assign_groups(c.groups);
  c.asg_tiles = c.groups / c.atg + c.nslot + 1;
  c.pack_tiles = c.groups / PACK_GROUPS + c.nslot + 1;
  for (uint32_t r = 0; r < n_req; r++) {
    const uint32_t a = h_rb ? h_rb[r] : 0, e = h_rb ? h_rb[r + 1] : nb;
    const uint64_t bytes = nb ? h_off[e] - h_off[a] : 0;
    c.max_words = std::max<uint64_t>(c.max_words, compress_bound(bytes, e - a) / 4);
  }
  return c;
}

// The compress workspace, carved in a fixed order (sizing and carving take
// the same path).
struct CWork {
  uint64_t *off_copy, *rout_copy;
  uint32_t* rb_copy;
  uint32_t *slot_base, *in_tile0, *cnt, *skip;
  uint64_t* in_rel;
  uint32_t *in_tile_blk, *in_tile_rs, *in_tile_out, *in_rle_n, *in_crc;
  void* in_rec;
  uint64_t* slot_in;
  uint32_t *slot_tile0, *slot_tile_blk, *tile_rs, *tile_out, *rle_n, *crc;
  void* rec;
  uint32_t *roff, *sort_tile0, *chunk0, *asg_tile0, *pack_tile0, *chunk_blk, *asg_blk, *pack_blk;
  uint64_t *sbase, *selb;
  uint8_t *text, *L;
  uint32_t* primary;
  uint16_t* syms;
  uint32_t *nsyms, *inuse, *freq;
  uint8_t *sel, *selmtf;
  uint64_t *gbits, *blkbit, *info;
  unsigned long long* gstate;
  BlockTables* tabs;
  void *hws, *stage;  // huffman scratch; sort / MTF scratch (shared: the sort's is free after bwt_out)
  size_t stage_bytes;
};

size_t carve_compress(char* base, const CBounds& c, uint32_t n_req, CWork& w, size_t total_cap) {
  Carve cv{base};
  const uint32_t ns = std::max<uint32_t>(c.nslot, 1);
  w.off_copy = cv.take<uint64_t>(c.nb + 1);
  w.rout_copy = cv.take<uint64_t>(n_req + 1);
  w.rb_copy = cv.take<uint32_t>(n_req + 1);
  w.slot_base = cv.take<uint32_t>(c.nb + 1);
  w.in_tile0 = cv.take<uint32_t>(c.nb + 1);
  w.cnt = cv.take<uint32_t>(PC_COUNT);
  w.skip = cv.take<uint32_t>(4);
  w.in_rel = cv.take<uint64_t>(c.nb + 1);
  const uint32_t it = c.direct ? 0 : c.in_tiles;
  w.in_tile_blk = cv.take<uint32_t>(it + 1);
  w.in_rec = cv.take<char>(rle_tile_bytes() * (it + 1));
  w.in_tile_rs = cv.take<uint32_t>(it + 1);
  w.in_tile_out = cv.take<uint32_t>(it + 1);
  w.in_rle_n = cv.take<uint32_t>(c.nb + 1);
  w.in_crc = cv.take<uint32_t>(c.nb + 1);
  w.slot_in = cv.take<uint64_t>(ns + 1);
  w.slot_tile0 = cv.take<uint32_t>(ns + 1);
  w.slot_tile_blk = cv.take<uint32_t>(c.slot_tiles + 1);
  w.rec = cv.take<char>(rle_tile_bytes() * (c.slot_tiles + 1));
  w.tile_rs = cv.take<uint32_t>(c.slot_tiles + 1);
  w.tile_out = cv.take<uint32_t>(c.slot_tiles + 1);
  w.rle_n = cv.take<uint32_t>(ns);
  w.crc = cv.take<uint32_t>(ns);
  w.roff = cv.take<uint32_t>(ns + 1);
  w.sbase = cv.take<uint64_t>(ns);
  w.selb = cv.take<uint64_t>(ns + 1);
  w.sort_tile0 = cv.take<uint32_t>(ns + 1);
  w.chunk0 = cv.take<uint32_t>(ns + 1);
  w.asg_tile0 = cv.take<uint32_t>(ns + 1);
  w.pack_tile0 = cv.take<uint32_t>(ns + 1);
  w.chunk_blk = cv.take<uint32_t>(c.chunks + 1);
  w.asg_blk = cv.take<uint32_t>(c.asg_tiles + 1);
  w.pack_blk = cv.take<uint32_t>(c.pack_tiles + 1);
  w.text = cv.take<uint8_t>((size_t)c.rows + 64);
  w.L = cv.take<uint8_t>((size_t)c.rows + 64);
  w.primary = cv.take<uint32_t>(ns);
  w.syms = cv.take<uint16_t>((size_t)c.rows + ns + 64);
  w.nsyms = cv.take<uint32_t>(ns);
  w.inuse = cv.take<uint32_t>((size_t)ns * 8);
  w.freq = cv.take<uint32_t>((size_t)ns * MAXA);
  w.sel = cv.take<uint8_t>((size_t)c.groups + 1);
  w.selmtf = cv.take<uint8_t>((size_t)c.groups + 1);
  w.gbits = cv.take<uint64_t>((size_t)c.groups + 1);
  w.gstate = cv.take<unsigned long long>(scan_lb_states(c.groups) + 1);
  w.tabs = cv.take<BlockTables>(ns);
  w.blkbit = cv.take<uint64_t>(ns);
  w.info = cv.take<uint64_t>(2 * (size_t)n_req + 2);
  w.hws = cv.take<char>(huff_workspace_bytes(ns));
  const size_t stage = std::max(bwt_workspace_bytes(c.rows, ns), mtf_workspace_bytes(c.rows, ns));
  w.stage = cv.take<char>(stage);
  w.stage_bytes = base ? total_cap - ((char*)w.stage - base) : stage;
  return cv.used + 256;
}

// The whole compressor for n_req streams: request r = input blocks
// [rb[r], rb[r+1]), written from byte rout[r] of d_out.  d_off / d_rb /
// d_rout are device tables (already in the workspace or the caller's).
int compress_enqueue(bzg_ctx* ctx, const CBounds& c, const CWork& w, const uint8_t* in, const uint64_t* d_off,
                     const uint32_t* d_rb, const uint64_t* d_rout, uint32_t n_req, int level, uint8_t* d_out,
                     uint64_t* d_out_bytes, uint32_t* d_n_blocks, hipStream_t st) {
  uint32_t* err = ctx->status;
  const uint32_t nb = c.nb, ns = c.nslot;
  HIPX(plan_input(d_off, nb, c.L, w.slot_base, w.in_tile0, w.cnt + PC_IN_TILES, w.in_rel, st));
  if (ns) {
    const uint64_t* slot_in = w.in_rel;
    if (!c.direct) {  // whole-block RLE1 lengths, then the cuts
      MapSet m{};
      m.map[0] = MapDesc{w.in_tile0, w.in_tile_blk, w.cnt + PC_IN_TILES, c.in_tiles, nb};
      m.nmaps = 1;
      m.err = err;
      HIPX(fill_maps(m, st));
      {
        ProfScope ps("rle1_tiles", st, 0, w.cnt + PC_IN_TILES, RLE_TILE);
        HIPX(rle1_tiles(in, persist_grid(c.in_tiles, ONE_TILE_EACH), w.cnt + PC_IN_TILES, w.in_tile_blk, w.in_tile0, w.in_rel,
                        ctx->crc_tab, ctx->crc_tab + CRC_POW_AT, w.in_rec, st));
      }
      HIPX(rle1_blocks(nb, w.in_tile0, w.in_rel, ctx->crc_tab + CRC_POW_AT, w.in_rec, w.in_tile_rs, w.in_tile_out,
                       w.in_rle_n, w.in_crc, st));
      HIPX(rle1_split(in, w.in_rel, nb, w.in_tile0, w.in_rec, w.in_tile_rs, w.in_tile_out, w.in_rle_n, w.slot_base,
                      ns, c.L, w.slot_in, err, st));
      slot_in = w.slot_in;
    }
    HIPX(plan_slot_tiles(slot_in, ns, w.slot_tile0, w.cnt + PC_RLE_TILES, st));
    {
      MapSet m{};
      m.map[0] = MapDesc{w.slot_tile0, w.slot_tile_blk, w.cnt + PC_RLE_TILES, c.slot_tiles, ns};
      m.nmaps = 1;
      m.err = err;
      HIPX(fill_maps(m, st));
    }
    {
      ProfScope ps("rle1_tiles", st, 0, w.cnt + PC_RLE_TILES, RLE_TILE);
      HIPX(rle1_tiles(in, persist_grid(c.slot_tiles, ONE_TILE_EACH), w.cnt + PC_RLE_TILES, w.slot_tile_blk, w.slot_tile0, slot_in,
                      ctx->crc_tab, ctx->crc_tab + CRC_POW_AT, w.rec, st));
    }
    HIPX(rle1_blocks(ns, w.slot_tile0, slot_in, ctx->crc_tab + CRC_POW_AT, w.rec, w.tile_rs, w.tile_out, w.rle_n,
                     w.crc, st));
    // the layout of every later stage, from the RLE1 lengths
    BwtWork bw;
    if (!bwt_carve(w.stage, w.stage_bytes, c.rows, ns, bw)) return fail(ctx, BZG_EINTERNAL, "sort workspace");
    {
      PlanArgs a{ns, c.mtf_ch, c.atg, 1};
      PlanOut o{w.roff, w.sbase, w.selb, w.sort_tile0, bw.segs[0], w.chunk0, w.asg_tile0, w.pack_tile0, w.cnt};
      HIPX(plan_layout(w.rle_n, nullptr, a, o, st));
      MapSet m{};
      m.map[0] = MapDesc{w.sort_tile0, bw.owner[0], w.cnt + PC_SORT_TILES, c.sort_tiles, ns};
      m.map[1] = MapDesc{w.chunk0, w.chunk_blk, w.cnt + PC_CHUNKS, c.chunks, ns};
      m.map[2] = MapDesc{w.asg_tile0, w.asg_blk, w.cnt + PC_ASSIGN_TILES, c.asg_tiles, ns};
      m.map[3] = MapDesc{w.pack_tile0, w.pack_blk, w.cnt + PC_PACK_TILES, c.pack_tiles, ns};
      m.nmaps = 4;
      m.err = err;
      HIPX(fill_maps(m, st));
    }
    {
      ProfScope ps("rle1_emit", st, 0, w.cnt + PC_RLE_TILES, RLE_TILE, w.cnt + PC_ROWS, 1.0);
      HIPX(rle1_emit(in, persist_grid(c.slot_tiles, ONE_TILE_EACH), w.cnt + PC_RLE_TILES, w.slot_tile_blk, w.slot_tile0, slot_in,
                     w.tile_rs, w.tile_out, w.roff, w.text, st));
    }
    // BWT
    BwtBounds bd{ns, c.rows, c.max_len, c.sort_tiles};
    HIPX(bwt_sort(bw, w.text, w.roff, w.cnt + PC_SORT_TILES, bd, err, nullptr, st));
    HIPX(bwt_output(w.text, w.roff, ns, w.cnt + PC_ROWS, c.rows, bw.SA, w.L, w.primary, nullptr, st));
    // MTF + RUNA/RUNB (the sort's scratch is free again)
    hipError_t e = mtf_run(w.L, w.roff, ns, c.rows, w.chunk_blk, w.chunk0, w.cnt + PC_CHUNKS, w.stage, w.stage_bytes,
                           w.syms, w.sbase, w.nsyms, w.inuse, w.freq, err, ctx->err, st);
    if (e != hipSuccess) return ctx->err.empty() ? hip_fail(ctx, e, "mtf") : BZG_EINTERNAL;
    // Huffman tables and group bit counts
    HuffArgs ha{};
    ha.nb = ns;
    ha.syms = w.syms;
    ha.sym_base = w.sbase;
    ha.nsyms = w.nsyms;
    ha.freq = w.freq;
    ha.inuse = w.inuse;
    ha.sel_base = w.selb;
    ha.sel = w.sel;
    ha.selmtf = w.selmtf;
    ha.gbits = w.gbits;
    ha.tabs = w.tabs;
    ha.err = err;
    ha.tile_blk = w.asg_blk;
    ha.blk_tile0 = w.asg_tile0;
    ha.n_tiles = w.cnt + PC_ASSIGN_TILES;
    ha.tiles_cap = c.asg_tiles;
    ha.tile_groups = c.atg;
    ha.ws = w.hws;
    ha.fixed = ctx->fixed_g ? ctx->fixed_tab : nullptr;
    ha.fixed_g = ctx->fixed_g;
    HIPX(huff_run(ha, st));
    {
      ProfScope ps("scan", st, 0, w.cnt + PC_GROUPS_LO, 16.0);
      HIPX(scan_lb_u64(w.gbits, w.cnt + PC_GROUPS_LO, c.groups, 1, w.gstate, err, persist_grid(scan_dev_tiles(c.groups), ONE_TILE_EACH),
                       st));
    }
  }
  // stream layout, sizes and the capacity check
  HIPX(pack_layout(ns, n_req, d_rb, d_rout, w.tabs, 0, nullptr, w.blkbit, w.crc, w.info, d_out_bytes, d_n_blocks,
                   w.slot_base, w.skip, err, st));
  {
    ProfScope ps("pack", st, 0, w.cnt + PC_ROWS, 2.0);  // symbols in (the streams out are not counted here)
    HIPX(zero_streams(n_req, c.max_words, d_rout, w.info, (uint32_t*)d_out, w.skip, st));
    HIPX(pack_run(ns, w.tabs, 0, w.blkbit, w.crc, w.primary, w.inuse, w.selb, w.sel, w.selmtf, w.gbits,
                  w.cnt + PC_PACK_TILES, c.pack_tiles, w.pack_blk, w.pack_tile0, w.syms, w.sbase, w.nsyms, level,
                  n_req, d_rout, w.info, (uint32_t*)d_out, w.skip, st));
  }
  return 0;
}

// Argument checks shared by compress_blocks and compress_batch.
int check_compress(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks, int level) {
  if (!h_offsets) return fail(ctx, BZG_EINVAL, "null h_offsets");
  if (level < 1 || level > 9) return fail(ctx, BZG_EINVAL, "level must be 1..9");
  if (n_blocks && !offsets_ok(h_offsets, n_blocks)) return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (n_blocks && h_offsets[n_blocks] > h_offsets[0] && !d_in) return fail(ctx, BZG_EINVAL, "null input");
  if (n_blocks && h_offsets[n_blocks] - h_offsets[0] >= (1ull << 31))
    return fail(ctx, BZG_EINVAL, "input too large for one call (2^31 bytes)");
  return 0;
}

int compress_common(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                    uint32_t n_blocks, const uint32_t* d_rb, const uint32_t* h_rb, uint32_t n_req, int level,
                    uint8_t* d_out, const uint64_t* d_rout, const uint64_t* h_rout, uint64_t out_cap,
                    uint64_t* d_out_bytes, uint32_t* d_n_blocks, void* d_ws, size_t ws_bytes, hipStream_t st) {
  HIPX(hipSetDevice(ctx->device));
  TuneGuard tg(ctx, h_offsets, n_blocks);
  const uint64_t zero_off = 0;
  const uint64_t* hoff = n_blocks ? h_offsets : &zero_off;
  const CBounds c = compress_bounds(hoff, n_blocks, level, h_rb, n_req);
  CWork w;
  const size_t need = carve_compress(nullptr, c, n_req, w, 0);
  void* ws;
  int rc = get_ws(ctx, d_ws, ws_bytes, need, st, &ws);
  if (rc) return rc;
  const size_t cap = d_ws ? ws_bytes : ctx->pool_cap;
  carve_compress((char*)ws, c, n_req, w, cap);
  // device tables: the caller's, or copies of the host ones
  const uint64_t* d_off = d_offsets;
  if (!d_off) {
    std::vector<uint64_t> tmp;
    if (!n_blocks) tmp.assign(1, 0);
    if ((rc = upload(ctx, {{w.off_copy, n_blocks ? h_offsets : tmp.data(), (size_t)(n_blocks + 1) * 8}}, st)))
      return rc;
    d_off = w.off_copy;
  }
  const uint8_t* in = d_in ? d_in + (n_blocks ? h_offsets[0] : 0) : nullptr;
  if (h_rb) {  // compress_batch: request tables
    if (!d_rb || !d_rout) {
      if ((rc = upload(ctx,
                       {{d_rb ? nullptr : (void*)w.rb_copy, h_rb, d_rb ? 0 : (size_t)(n_req + 1) * 4},
                        {d_rout ? nullptr : (void*)w.rout_copy, h_rout, d_rout ? 0 : (size_t)(n_req + 1) * 8}},
                       st)))
        return rc;
      if (!d_rb) d_rb = w.rb_copy;
      if (!d_rout) d_rout = w.rout_copy;
    }
    HIPX(call_init(w.skip, nullptr, 0, nullptr, 0, st));
  } else {  // compress_blocks: one request over every block, d_out[0, cap)
    HIPX(call_init(w.skip, w.rb_copy, n_blocks, w.rout_copy, out_cap & ~3ull, st));
    d_rb = w.rb_copy;
    d_rout = w.rout_copy;
  }
  rc = compress_enqueue(ctx, c, w, in, d_off, d_rb, d_rout, n_req, level, d_out, d_out_bytes, d_n_blocks, st);
  if (rc) return rc;
  return end_ws(ctx, d_ws, st);
}

// The device-side error flags of the calls so far (the work that set them
// has completed), as a return code; the flags are cleared.
int status_result(bzg_ctx* ctx) {
  uint32_t s[4];
  HIPX(hipMemcpy(s, ctx->status, sizeof(s), hipMemcpyDeviceToHost));
  if (!s[0]) return 0;
  HIPX(hipMemset(ctx->status, 0, sizeof(s)));
  if (s[0] & ERR_BOUND) return fail(ctx, BZG_EINTERNAL, "a device-side count passed its bound; results are not valid");
  if (s[0] & ERR_STREAM)
    return fail(ctx, BZG_EDATA, "a compressed stream does not decode (corrupt, or a form this decoder does not read)");
  if (s[0] & ERR_SYMBOL)
    return fail(ctx, BZG_EDATA, "a symbol outside its block's alphabet (or more symbols than the block's capacity)");
  return fail(ctx, BZG_ECAPACITY, "an output range was too small; nothing was packed");
}

// Tune cache: a JSON object, one entry per line,
//   "<arch>|<HIP runtime version>|<bucket>": {"mtf_chunk": M, "assign_groups": A, "count_steps": C, "ms": T},
// where bucket = floor(log2 bytes) * 256 + floor(log2 blocks).  Entries of
// other devices and runtimes are kept in the file but not used.
void load_tune_cache(bzg_ctx* ctx) {
  std::ifstream f(ctx->tune_path);
  std::string line;
  while (std::getline(f, line)) {
    char key[256];
    unsigned m = 0, a = 0, c = 0;
    if (sscanf(line.c_str(), " \"%255[^\"]\": {\"mtf_chunk\": %u, \"assign_groups\": %u, \"count_steps\": %u", key, &m,
               &a, &c) != 4)
      continue;
    const std::string k = key;
    const size_t bar = k.rfind('|');
    if (bar == std::string::npos || k.substr(0, bar) != ctx->tune_id) continue;
    Tune t;
    t.mtf_chunk = m;
    t.assign_groups = a;
    t.count_steps = c;
    ctx->tune_table[(uint32_t)std::stoul(k.substr(bar + 1))] = t;
  }
}

int save_tune_entry(bzg_ctx* ctx, uint32_t bucket, const Tune& t, double ms) {
  std::vector<std::string> lines;
  {
    std::ifstream f(ctx->tune_path);
    std::string line;
    while (std::getline(f, line))
      if (line.find("\"mtf_chunk\"") != std::string::npos) {
        while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
        lines.push_back(line);
      }
  }
  const std::string key = ctx->tune_id + "|" + std::to_string(bucket);
  char buf[512];
  snprintf(buf, sizeof(buf), "  \"%s\": {\"mtf_chunk\": %u, \"assign_groups\": %u, \"count_steps\": %u, \"ms\": %.4f}",
           key.c_str(), t.mtf_chunk, t.assign_groups, t.count_steps, ms);
  bool replaced = false;
  for (std::string& l : lines)
    if (l.find("\"" + key + "\"") != std::string::npos) {
      l = buf;
      replaced = true;
    }
  if (!replaced) lines.push_back(buf);
  std::ofstream o(ctx->tune_path, std::ios::trunc);
  if (!o) return fail(ctx, BZG_EINVAL, "cannot write the tune cache " + ctx->tune_path);
  o << "{\n";
  for (size_t i = 0; i < lines.size(); i++) o << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
  o << "}\n";
  return 0;
}

}  // namespace

extern "C" {

int bzg_create(bzg_ctx** out, int hip_device, const char* tune_cache_path) {
  if (!out) return BZG_EINVAL;
  *out = nullptr;
  bzg_ctx* ctx = new (std::nothrow) bzg_ctx();
  if (!ctx) return BZG_ENOMEM;
  ctx->device = hip_device;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = hipMalloc(&ctx->crc_tab, CRC_TAB_WORDS * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&ctx->status, 256);
  if (e == hipSuccess) e = hipMemset(ctx->status, 0, 256);
  if (e == hipSuccess) {
    uint32_t h[CRC_TAB_WORDS];
    crc_tables(h, h + CRC_POW_AT);
    e = hipMemcpy(ctx->crc_tab, h, sizeof(h), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->pool_ev, hipEventDisableTiming);
  for (int h = 0; h < 2 && e == hipSuccess; h++) e = hipEventCreateWithFlags(&ctx->stage_ev[h], hipEventDisableTiming);
  if (e == hipSuccess) {
    ctx->stage_half = 1 << 19;
    e = hipHostMalloc((void**)&ctx->stage, 2 * ctx->stage_half, hipHostMallocDefault);
  }
  if (e == hipSuccess) e = hipGetSymbolAddress(&ctx->scratch, HIP_SYMBOL(scratch));
  if (e == hipSuccess) bwt_warm_grids();  // grid sizes cached now, so later calls compute none
  if (e != hipSuccess) {
    bzg_destroy(ctx);
    return BZG_EHIP;
  }
  {
    hipDeviceProp_t prop{};
    int rv = 0;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && hipRuntimeGetVersion(&rv) == hipSuccess) {
      std::string arch = prop.gcnArchName;
      arch = arch.substr(0, arch.find(':'));
      ctx->tune_id = arch + "|" + std::to_string(rv);
    }
    (void)hipGetLastError();
  }
  if (tune_cache_path && *tune_cache_path) {
    ctx->tune_path = tune_cache_path;
    load_tune_cache(ctx);
  }
  *out = ctx;
  return 0;
}

void bzg_destroy(bzg_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->pool) {
    (void)hipFreeAsync(ctx->pool, nullptr);
    (void)hipDeviceSynchronize();
  }
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  if (ctx->crc_tab) (void)hipFree(ctx->crc_tab);
  if (ctx->fixed_tab) (void)hipFree(ctx->fixed_tab);
  if (ctx->status) (void)hipFree(ctx->status);
  if (ctx->prof.slots) (void)hipFree(ctx->prof.slots);
  if (ctx->pool_ev) (void)hipEventDestroy(ctx->pool_ev);
  for (int h = 0; h < 2; h++)
    if (ctx->stage_ev[h]) (void)hipEventDestroy(ctx->stage_ev[h]);
  for (auto& p : ctx->prof.pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  bzg_ctx::HostIo& h = ctx->hio;
  for (int b = 0; b < 2; b++) {
    if (h.din[b]) (void)hipFree(h.din[b]);
    if (h.dout[b]) (void)hipFree(h.dout[b]);
    if (h.pin[b]) (void)hipHostFree(h.pin[b]);
    for (hipEvent_t e : {h.in_ev[b], h.comp_ev[b], h.out_ev[b]})
      if (e) (void)hipEventDestroy(e);
  }
  if (h.dsize) (void)hipFree(h.dsize);
  if (h.hsize) (void)hipHostFree(h.hsize);
  if (h.up) (void)hipStreamDestroy(h.up);
  if (h.down) (void)hipStreamDestroy(h.down);
  for (hipStream_t q : ctx->dec_side)
    if (q) (void)hipStreamDestroy(q);
  for (hipEvent_t e : {ctx->dec_fork, ctx->dec_join[0], ctx->dec_join[1]})
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

const char* bzg_last_error(const bzg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int bzg_check(bzg_ctx* ctx, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  HIPX(hipSetDevice(ctx->device));
  HIPX(hipStreamSynchronize((hipStream_t)stream));
  return status_result(ctx);
}

int bzg_set_fixed_tables(bzg_ctx* ctx, const uint8_t* h_lens, int n_tables) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  if (n_tables == 0) {
    ctx->fixed_g = 0;
    return 0;
  }
  if (n_tables < 2 || n_tables > MAXG || !h_lens) return fail(ctx, BZG_EINVAL, "2..6 tables of 258 lengths");
  for (int t = 0; t < n_tables; t++) {
    uint64_t kraft = 0;  // in units of 2^-MAXLEN
    for (int v = 0; v < MAXA; v++) {
      const int l = h_lens[t * MAXA + v];
      if (l < 1 || l > MAXLEN) return fail(ctx, BZG_EINVAL, "code lengths must be 1..17");
      kraft += 1ull << (MAXLEN - l);
    }
    if (kraft > (1ull << MAXLEN))
      return fail(ctx, BZG_EINVAL, "table " + std::to_string(t) + " is not a prefix code (Kraft sum above 1)");
  }
  HIPX(hipSetDevice(ctx->device));
  if (!ctx->fixed_tab) HIPX(hipMalloc((void**)&ctx->fixed_tab, MAXG * MAXA));
  // synchronous: earlier calls that read the old tables have completed first
  HIPX(hipDeviceSynchronize());
  HIPX(hipMemcpy(ctx->fixed_tab, h_lens, (size_t)n_tables * MAXA, hipMemcpyHostToDevice));
  ctx->fixed_g = n_tables;
  return 0;
}

int bzg_profile(bzg_ctx* ctx, int enable) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (enable) {
    ctx->prof.acc.clear();
    if (!ctx->prof.slots) {
      ctx->prof.nslots = 1 << 18;
      HIPX(hipMalloc(&ctx->prof.slots, (size_t)ctx->prof.nslots * 4));
    }
  }
  ctx->prof.on = enable != 0;
  return 0;
}

int bzg_profile_read(bzg_ctx* ctx, char* buf, size_t cap) {
  if (!ctx || !buf || cap == 0) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->prof.collect();
  std::string s;
  char line[256];
  for (auto& kv : ctx->prof.acc) {
    snprintf(line, sizeof(line), "%s %llu %.6f %.1f\n", kv.first.c_str(), (unsigned long long)kv.second.launches,
             kv.second.ms, kv.second.bytes);
    s += line;
  }
  if (s.size() + 1 > cap) return fail(ctx, BZG_ECAPACITY, "profile text needs " + std::to_string(s.size() + 1));
  memcpy(buf, s.c_str(), s.size() + 1);
  return 0;
}

uint64_t bzg_compress_bound(uint64_t n_bytes, uint32_t n_blocks) { return compress_bound(n_bytes, n_blocks); }

}  // extern "C"

namespace {

// ------------------------------------------------------------ BWT / MTF / Huffman calls

struct SWork {  // the per-stage calls' workspace
  uint64_t* off_copy;
  uint64_t* out_copy;
  uint32_t *roff, *sort_tile0, *chunk0, *chunk_blk, *asg_tile0, *asg_blk, *pack_tile0, *pack_blk, *cnt, *skip;
  uint64_t *sbase, *selb;
  uint32_t *freq, *ns_eff;
  uint8_t *sel, *selmtf;
  uint64_t *gbits, *blkbit;
  unsigned long long* gstate;
  BlockTables* tabs;
  void *hws, *stage;
  size_t stage_bytes;
};

struct SBounds {
  uint32_t nb = 0, rows = 0, max_len = 0, sort_tiles = 0, mtf_ch = 0, chunks = 0, groups = 0, atg = 0, asg_tiles = 0,
           pack_tiles = 0;
};

SBounds stage_bounds(const uint64_t* h_off, uint32_t nb, int call) {
  SBounds b;
  b.nb = nb;
  uint64_t rows = nb ? h_off[nb] - h_off[0] : 0;
  b.rows = (uint32_t)std::min<uint64_t>(rows, 0xFFFFFFF0ull);
  for (uint32_t k = 0; k < nb; k++) b.max_len = (uint32_t)std::max<uint64_t>(b.max_len, h_off[k + 1] - h_off[k]);
  b.sort_tiles = b.rows / RADIX_TILE + nb + 1;
  b.mtf_ch = mtf_chunk_rows(b.rows, nb);
  b.chunks = b.rows / b.mtf_ch + nb + 1;
  if (call == BZG_CALL_HUFFMAN) {
    uint64_t g = 0;
    for (uint32_t k = 0; k < nb; k++) g += (h_off[k + 1] - h_off[k] + GROUP - 1) / GROUP;
    b.groups = (uint32_t)g + 1;
    b.atg = huff_assign_groups(g);
    b.asg_tiles = b.groups / b.atg + nb + 1;
    b.pack_tiles = b.groups / PACK_GROUPS + nb + 1;
  }
  return b;
}

size_t carve_stage(char* base, const SBounds& b, int call, SWork& w, size_t total_cap) {
  Carve cv{base};
  const uint32_t nb = std::max<uint32_t>(b.nb, 1);
  w.off_copy = cv.take<uint64_t>(nb + 1);
  w.out_copy = cv.take<uint64_t>(nb + 1);
  w.cnt = cv.take<uint32_t>(PC_COUNT);
  w.skip = cv.take<uint32_t>(4);
  w.roff = cv.take<uint32_t>(nb + 1);
  w.sbase = cv.take<uint64_t>(nb);
  w.sort_tile0 = cv.take<uint32_t>(nb + 1);
  w.chunk0 = cv.take<uint32_t>(nb + 1);
  w.chunk_blk = cv.take<uint32_t>(call == BZG_CALL_MTF ? b.chunks + 1 : 1);
  // symbol counts per block: written by the MTF stage, read by the Huffman one
  w.freq = cv.take<uint32_t>(call == BZG_CALL_HUFFMAN || call == BZG_CALL_MTF ? (size_t)nb * MAXA : 1);
  w.ns_eff = cv.take<uint32_t>(nb);
  w.selb = cv.take<uint64_t>(nb + 1);
  w.asg_tile0 = cv.take<uint32_t>(nb + 1);
  w.pack_tile0 = cv.take<uint32_t>(nb + 1);
  w.asg_blk = cv.take<uint32_t>(b.asg_tiles + 1);
  w.pack_blk = cv.take<uint32_t>(b.pack_tiles + 1);
  w.sel = cv.take<uint8_t>(b.groups + 1);
  w.selmtf = cv.take<uint8_t>(b.groups + 1);
  w.gbits = cv.take<uint64_t>(b.groups + 1);
  w.gstate = cv.take<unsigned long long>(scan_lb_states(b.groups) + 1);
  w.blkbit = cv.take<uint64_t>(nb);
  w.tabs = cv.take<BlockTables>(call == BZG_CALL_HUFFMAN ? nb : 1);
  w.hws = cv.take<char>(call == BZG_CALL_HUFFMAN ? huff_workspace_bytes(nb) : 1);
  size_t stage = 256;
  if (call == BZG_CALL_BWT) stage = bwt_workspace_bytes(b.rows, nb);
  if (call == BZG_CALL_MTF) stage = mtf_workspace_bytes(b.rows, nb);
  w.stage = cv.take<char>(stage);
  w.stage_bytes = base ? total_cap - ((char*)w.stage - base) : stage;
  return cv.used + 256;
}

int stage_prologue(bzg_ctx* ctx, int call, const uint64_t* h_off, uint32_t nb, const uint64_t* d_off_in,
                   void* d_ws, size_t ws_bytes, hipStream_t st, SBounds& b, SWork& w, const uint64_t** d_off) {
  HIPX(hipSetDevice(ctx->device));
  b = stage_bounds(h_off, nb, call);
  const size_t need = carve_stage(nullptr, b, call, w, 0);
  void* ws;
  int rc = get_ws(ctx, d_ws, ws_bytes, need, st, &ws);
  if (rc) return rc;
  carve_stage((char*)ws, b, call, w, d_ws ? ws_bytes : ctx->pool_cap);
  *d_off = d_off_in;
  if (!d_off_in) {
    if ((rc = upload(ctx, {{w.off_copy, h_off, (size_t)(nb + 1) * 8}}, st))) return rc;
    *d_off = w.off_copy;
  }
  return 0;
}

int check_blocks(bzg_ctx* ctx, const uint64_t* h_offsets, uint32_t n_blocks) {
  if (!offsets_ok(h_offsets, n_blocks)) return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (h_offsets[n_blocks] - h_offsets[0] >= (1ull << 32) - 4096) return fail(ctx, BZG_EINVAL, "batch too large");
  for (uint32_t k = 0; k < n_blocks; k++) {
    const uint64_t n = h_offsets[k + 1] - h_offsets[k];
    if (n == 0 || n > BZG_MAX_BLOCK) return fail(ctx, BZG_EINVAL, "block length outside 1..BZG_MAX_BLOCK");
  }
  return 0;
}

}  // namespace

extern "C" {

int bzg_workspace_size(bzg_ctx* ctx, int call, const uint64_t* h_offsets, uint32_t n_blocks, int level,
                       uint32_t n_req, size_t* bytes) {
  if (!ctx || !bytes || !h_offsets) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  TuneGuard tg(ctx, h_offsets, n_blocks);
  if (n_blocks && !offsets_ok(h_offsets, n_blocks)) return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (call == BZG_CALL_COMPRESS) {
    if (level < 1 || level > 9) return fail(ctx, BZG_EINVAL, "level must be 1..9");
    if (n_req == 0) n_req = 1;
    // the request split does not change the bound but for the stream words
    const CBounds c = compress_bounds(h_offsets, n_blocks, level, nullptr, 1);
    CWork w;
    *bytes = carve_compress(nullptr, c, n_req, w, 0);
    return 0;
  }
  if (call != BZG_CALL_BWT && call != BZG_CALL_MTF && call != BZG_CALL_HUFFMAN)
    return fail(ctx, BZG_EINVAL, "unknown call id");
  SBounds b = stage_bounds(h_offsets, n_blocks, call);
  SWork w;
  *bytes = carve_stage(nullptr, b, call, w, 0);
  return 0;
}

int bwt_forward_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                      uint32_t n_blocks, uint8_t* d_bwt, uint32_t* d_primary, uint32_t* d_sa, void* d_ws,
                      size_t ws_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  TuneGuard tg(ctx, h_offsets, n_blocks);
  ProfGuard pg(ctx);
  if (!h_offsets || !d_bwt || !d_primary || (n_blocks && !d_in)) return fail(ctx, BZG_EINVAL, "null pointer");
  if (n_blocks == 0) return 0;
  int rc = check_blocks(ctx, h_offsets, n_blocks);
  if (rc) return rc;
  if ((uintptr_t)(d_in + h_offsets[0]) & 3) return fail(ctx, BZG_EINVAL, "d_in + h_offsets[0] must be 4-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  SBounds b;
  SWork w;
  const uint64_t* d_off;
  if ((rc = stage_prologue(ctx, BZG_CALL_BWT, h_offsets, n_blocks, d_offsets, d_ws, ws_bytes, st, b, w, &d_off)))
    return rc;
  BwtWork bw;
  if (!bwt_carve(w.stage, w.stage_bytes, b.rows, n_blocks, bw)) return fail(ctx, BZG_EINTERNAL, "sort workspace");
  PlanArgs a{n_blocks, b.mtf_ch, 1, 0};
  PlanOut o{w.roff, nullptr, nullptr, w.sort_tile0, bw.segs[0], nullptr, nullptr, nullptr, w.cnt};
  HIPX(plan_layout(nullptr, d_off, a, o, st));
  MapSet m{};
  m.map[0] = MapDesc{w.sort_tile0, bw.owner[0], w.cnt + PC_SORT_TILES, b.sort_tiles, n_blocks};
  m.nmaps = 1;
  m.err = ctx->status;
  HIPX(fill_maps(m, st));
  const uint8_t* text = d_in + h_offsets[0];
  BwtBounds bd{n_blocks, b.rows, b.max_len, b.sort_tiles};
  HIPX(bwt_sort(bw, text, w.roff, w.cnt + PC_SORT_TILES, bd, ctx->status, nullptr, st));
  HIPX(bwt_output(text, w.roff, n_blocks, w.cnt + PC_ROWS, b.rows, bw.SA, d_bwt + h_offsets[0], d_primary,
                  d_sa ? d_sa + h_offsets[0] : nullptr, st));
  return end_ws(ctx, d_ws, st);
}

int mtf_encode_batch(bzg_ctx* ctx, const uint8_t* d_bwt, const uint64_t* d_offsets, const uint64_t* h_offsets,
                     uint32_t n_blocks, uint16_t* d_syms, uint32_t* d_nsyms, uint8_t* d_inuse, void* d_ws,
                     size_t ws_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  TuneGuard tg(ctx, h_offsets, n_blocks);
  ProfGuard pg(ctx);
  if (!h_offsets || !d_syms || !d_nsyms || !d_inuse || (n_blocks && !d_bwt))
    return fail(ctx, BZG_EINVAL, "null pointer");
  if (n_blocks == 0) return 0;
  int rc = check_blocks(ctx, h_offsets, n_blocks);
  if (rc) return rc;
  if (((uintptr_t)d_inuse & 3) != 0) return fail(ctx, BZG_EINVAL, "d_inuse must be 4-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  SBounds b;
  SWork w;
  const uint64_t* d_off;
  if ((rc = stage_prologue(ctx, BZG_CALL_MTF, h_offsets, n_blocks, d_offsets, d_ws, ws_bytes, st, b, w, &d_off)))
    return rc;
  PlanArgs a{n_blocks, b.mtf_ch, 1, 0};
  PlanOut o{w.roff, w.sbase, nullptr, nullptr, nullptr, w.chunk0, nullptr, nullptr, w.cnt};
  HIPX(plan_layout(nullptr, d_off, a, o, st));
  MapSet m{};
  m.map[0] = MapDesc{w.chunk0, w.chunk_blk, w.cnt + PC_CHUNKS, b.chunks, n_blocks};
  m.nmaps = 1;
  m.err = ctx->status;
  HIPX(fill_maps(m, st));
  // syms + h_offsets[0]: block k's symbols at (relative offset) + k
  hipError_t e = mtf_run(d_bwt + h_offsets[0], w.roff, n_blocks, b.rows, w.chunk_blk, w.chunk0, w.cnt + PC_CHUNKS,
                         w.stage, w.stage_bytes, d_syms + h_offsets[0], w.sbase, d_nsyms, (uint32_t*)d_inuse, w.freq,
                         ctx->status, ctx->err, st);
  if (e != hipSuccess) return ctx->err.empty() ? hip_fail(ctx, e, "mtf") : BZG_EINTERNAL;
  return end_ws(ctx, d_ws, st);
}

int huffman_encode_batch(bzg_ctx* ctx, const uint16_t* d_syms, const uint32_t* d_nsyms, const uint8_t* d_inuse,
                         const uint64_t* d_sym_offsets, const uint64_t* h_sym_offsets, uint32_t n_blocks,
                         uint8_t* d_out, const uint64_t* d_out_offsets, const uint64_t* h_out_offsets,
                         uint64_t* d_nbits, uint8_t* d_tables, void* d_ws, size_t ws_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  TuneGuard tg(ctx, h_sym_offsets, n_blocks);
  ProfGuard pg(ctx);
  if (!h_sym_offsets || !h_out_offsets || !d_nbits || (n_blocks && (!d_syms || !d_nsyms || !d_inuse || !d_out)))
    return fail(ctx, BZG_EINVAL, "null pointer");
  if (n_blocks == 0) return 0;
  if (!offsets_ok(h_sym_offsets, n_blocks) || !offsets_ok(h_out_offsets, n_blocks))
    return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (((uintptr_t)d_out & 3) || (h_out_offsets[n_blocks] & 3) || (h_out_offsets[0] & 3) || ((uintptr_t)d_inuse & 3))
    return fail(ctx, BZG_EINVAL, "d_out/d_inuse must be 4-byte aligned and the output range multiples of 4");
  for (uint32_t k = 0; k < n_blocks; k++)
    if (h_sym_offsets[k + 1] - h_sym_offsets[k] > 2ull * BZG_MAX_BLOCK + 2)
      return fail(ctx, BZG_EINVAL, "symbol capacity per block too large");
  hipStream_t st = (hipStream_t)stream;
  SBounds b;
  SWork w;
  const uint64_t* d_soff;
  int rc;
  if ((rc = stage_prologue(ctx, BZG_CALL_HUFFMAN, h_sym_offsets, n_blocks, d_sym_offsets, d_ws, ws_bytes, st, b, w,
                           &d_soff)))
    return rc;
  const uint64_t* d_oo = d_out_offsets;
  if (!d_oo) {
    if ((rc = upload(ctx, {{w.out_copy, h_out_offsets, (size_t)(n_blocks + 1) * 8}}, st))) return rc;
    d_oo = w.out_copy;
  }
  HIPX(call_init(w.skip, nullptr, 0, nullptr, 0, st));
  PlanArgs a{n_blocks, b.mtf_ch, b.atg, 0};
  PlanOut o{nullptr, nullptr, w.selb, nullptr, nullptr, nullptr, w.asg_tile0, w.pack_tile0, w.cnt};
  HIPX(plan_layout(nullptr, d_soff, a, o, st));
  MapSet m{};
  m.map[0] = MapDesc{w.asg_tile0, w.asg_blk, w.cnt + PC_ASSIGN_TILES, b.asg_tiles, n_blocks};
  m.map[1] = MapDesc{w.pack_tile0, w.pack_blk, w.cnt + PC_PACK_TILES, b.pack_tiles, n_blocks};
  m.nmaps = 2;
  m.err = ctx->status;
  HIPX(fill_maps(m, st));
  HuffArgs ha{};
  ha.nb = n_blocks;
  ha.syms = d_syms;
  ha.sym_base = d_soff;
  ha.nsyms = d_nsyms;
  ha.freq = w.freq;
  ha.inuse = (const uint32_t*)d_inuse;
  ha.sel_base = w.selb;
  ha.sel = w.sel;
  ha.selmtf = w.selmtf;
  ha.gbits = w.gbits;
  ha.tabs = w.tabs;
  ha.err = ctx->status;
  ha.tile_blk = w.asg_blk;
  ha.blk_tile0 = w.asg_tile0;
  ha.n_tiles = w.cnt + PC_ASSIGN_TILES;
  ha.tiles_cap = b.asg_tiles;
  ha.tile_groups = b.atg;
  ha.ws = w.hws;
  ha.count_freq = true;
  ha.sym_off = d_soff;
  ha.ns_eff = w.ns_eff;
  ha.fixed = ctx->fixed_g ? ctx->fixed_tab : nullptr;
  ha.fixed_g = ctx->fixed_g;
  HIPX(huff_run(ha, st));
  HIPX(scan_lb_u64(w.gbits, w.cnt + PC_GROUPS_LO, b.groups, 1, w.gstate, ctx->status,
                   persist_grid(scan_dev_tiles(b.groups), ONE_TILE_EACH), st));
  HIPX(pack_layout(n_blocks, 1, nullptr, nullptr, w.tabs, 1, d_oo, w.blkbit, nullptr, d_nbits, nullptr, nullptr,
                   nullptr, w.skip, ctx->status, st));
  HIPX(zero_range((uint32_t*)(d_out + h_out_offsets[0]), (h_out_offsets[n_blocks] - h_out_offsets[0]) / 4, w.skip,
                  st));
  HIPX(pack_run(n_blocks, w.tabs, 1, w.blkbit, nullptr, nullptr, (const uint32_t*)d_inuse, w.selb, w.sel, w.selmtf,
                w.gbits, w.cnt + PC_PACK_TILES, b.pack_tiles, w.pack_blk, w.pack_tile0, d_syms, d_soff, w.ns_eff, 9, 0,
                nullptr, nullptr, (uint32_t*)d_out, w.skip, st));
  if (d_tables) HIPX(tables_export(n_blocks, w.tabs, d_tables, st));
  return end_ws(ctx, d_ws, st);
}

int compress_blocks(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                    uint32_t n_blocks, int level, uint8_t* d_out, uint64_t out_cap, uint64_t* d_out_bytes,
                    uint32_t* d_n_blocks, void* d_ws, size_t ws_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!d_out || !d_out_bytes) return fail(ctx, BZG_EINVAL, "null pointer");
  int rc = check_compress(ctx, d_in, h_offsets, n_blocks, level);
  if (rc) return rc;
  if ((uintptr_t)d_out & 3) return fail(ctx, BZG_EINVAL, "d_out must be 4-byte aligned");
  return compress_common(ctx, d_in, d_offsets, h_offsets, n_blocks, nullptr, nullptr, 1, level, d_out, nullptr,
                         nullptr, out_cap, d_out_bytes, d_n_blocks, d_ws, ws_bytes, (hipStream_t)stream);
}

int compress_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                   uint32_t n_blocks, const uint32_t* d_req_blocks, const uint32_t* h_req_blocks, uint32_t n_req,
                   int level, uint8_t* d_out, const uint64_t* d_out_offsets, const uint64_t* h_out_offsets,
                   uint64_t* d_out_bytes, void* d_ws, size_t ws_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!h_req_blocks || !h_out_offsets || !d_out_bytes || (n_req && !d_out))
    return fail(ctx, BZG_EINVAL, "null pointer");
  int rc = check_compress(ctx, d_in, h_offsets, n_blocks, level);
  if (rc) return rc;
  if (n_req > 65535) return fail(ctx, BZG_EINVAL, "at most 65535 requests per call");
  if (h_req_blocks[0] != 0 || h_req_blocks[n_req] != n_blocks)
    return fail(ctx, BZG_EINVAL, "request block ranges must start at 0 and end at n_blocks");
  for (uint32_t r = 0; r < n_req; r++) {
    if (h_req_blocks[r + 1] < h_req_blocks[r]) return fail(ctx, BZG_EINVAL, "request block ranges decrease");
    if (h_out_offsets[r + 1] < h_out_offsets[r]) return fail(ctx, BZG_EINVAL, "output offsets decrease");
  }
  for (uint32_t r = 0; r <= n_req; r++)
    if (h_out_offsets[r] & 3) return fail(ctx, BZG_EINVAL, "output offsets must be multiples of 4");
  if ((uintptr_t)d_out & 3) return fail(ctx, BZG_EINVAL, "d_out must be 4-byte aligned");
  if (n_req == 0) return 0;
  return compress_common(ctx, d_in, d_offsets, h_offsets, n_blocks, d_req_blocks, h_req_blocks, n_req, level, d_out,
                         d_out_offsets, h_out_offsets, 0, d_out_bytes, nullptr, d_ws, ws_bytes,
                         (hipStream_t)stream);
}

int compress_blocks_noalloc(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                            uint32_t n_blocks, int level, uint8_t* d_out, uint64_t out_cap, uint64_t* d_out_bytes,
                            uint32_t* d_n_blocks, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  TuneGuard tg(ctx, h_offsets, n_blocks);
  if (!d_out || !d_out_bytes || !d_offsets) return fail(ctx, BZG_EINVAL, "null pointer (d_offsets is required)");
  int rc = check_compress(ctx, d_in, h_offsets, n_blocks, level);
  if (rc) return rc;
  if ((uintptr_t)d_out & 3) return fail(ctx, BZG_EINVAL, "d_out must be 4-byte aligned");
  const uint64_t zero_off = 0;
  const CBounds c = compress_bounds(n_blocks ? h_offsets : &zero_off, n_blocks, level, nullptr, 1);
  CWork w;
  const size_t need = carve_compress(nullptr, c, 1, w, 0);
  if (need > SCRATCH_BYTES)
    return fail(ctx, BZG_EWORKSPACE, "the call needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                         std::to_string(SCRATCH_BYTES));
  // no profiling scopes here: they create events
  return compress_common(ctx, d_in, d_offsets, h_offsets, n_blocks, nullptr, nullptr, 1, level, d_out, nullptr,
                         nullptr, out_cap, d_out_bytes, d_n_blocks, ctx->scratch, SCRATCH_BYTES, (hipStream_t)stream);
}


}  // extern "C"

// ------------------------------------------------ input in host memory

namespace {

bool is_pinned(const void* p) {
  hipPointerAttribute_t a{};
  const bool ok = hipPointerGetAttributes(&a, p) == hipSuccess && a.type == hipMemoryTypeHost;
  (void)hipGetLastError();  // pageable memory may leave an error behind
  return ok;
}

// The buffers of compress_host for chunks of `in_bytes` input and
// `out_bytes` output (grown when too small; the old ones are idle then,
// since every call ends synchronised).
int hio_reserve(bzg_ctx* ctx, size_t in_bytes, size_t out_bytes, bool pin) {
  bzg_ctx::HostIo& h = ctx->hio;
  if (!h.up) {
    HIPX(hipStreamCreateWithFlags(&h.up, hipStreamNonBlocking));
    HIPX(hipStreamCreateWithFlags(&h.down, hipStreamNonBlocking));
    for (int b = 0; b < 2; b++) {
      HIPX(hipEventCreateWithFlags(&h.in_ev[b], hipEventDisableTiming));
      HIPX(hipEventCreateWithFlags(&h.comp_ev[b], hipEventDisableTiming));
      HIPX(hipEventCreateWithFlags(&h.out_ev[b], hipEventDisableTiming));
    }
    HIPX(hipMalloc((void**)&h.dsize, 2 * sizeof(uint64_t)));
    HIPX(hipHostMalloc((void**)&h.hsize, 2 * sizeof(uint64_t), hipHostMallocDefault));
  }
  for (int b = 0; b < 2; b++) {
    if (h.in_cap < in_bytes) {
      if (h.din[b]) HIPX(hipFree(h.din[b]));
      h.din[b] = nullptr;
      if (hipMalloc((void**)&h.din[b], in_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, BZG_ENOMEM, "device input buffer");
      }
    }
    if (h.out_cap < out_bytes) {
      if (h.dout[b]) HIPX(hipFree(h.dout[b]));
      h.dout[b] = nullptr;
      if (hipMalloc((void**)&h.dout[b], out_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, BZG_ENOMEM, "device output buffer");
      }
    }
    if (pin && h.pin_cap < in_bytes) {
      if (h.pin[b]) HIPX(hipHostFree(h.pin[b]));
      h.pin[b] = nullptr;
      if (hipHostMalloc((void**)&h.pin[b], in_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, BZG_ENOMEM, "pinned input buffer");
      }
    }
  }
  h.in_cap = std::max(h.in_cap, in_bytes);
  h.out_cap = std::max(h.out_cap, out_bytes);
  if (pin) h.pin_cap = std::max(h.pin_cap, in_bytes);
  return 0;
}

}  // namespace

extern "C" {

int compress_host(bzg_ctx* ctx, const uint8_t* h_in, uint64_t n_bytes, uint32_t block_bytes, int level,
                  uint64_t chunk_bytes, uint8_t* h_out, uint64_t out_cap, uint64_t* h_out_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!h_out || !h_out_bytes || (n_bytes && !h_in)) return fail(ctx, BZG_EINVAL, "null pointer");
  if (level < 1 || level > 9) return fail(ctx, BZG_EINVAL, "level must be 1..9");
  if (block_bytes == 0) block_bytes = 100000u * (uint32_t)level;
  uint64_t per = chunk_bytes ? chunk_bytes / block_bytes : 128;  // blocks per chunk
  if (per == 0) per = 1;
  const uint64_t cb = per * block_bytes;
  if (cb >= (1ull << 31)) return fail(ctx, BZG_EINVAL, "a chunk must hold less than 2^31 bytes");
  HIPX(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nc = n_bytes ? (n_bytes + cb - 1) / cb : 1;  // an empty input gives one empty stream
  const uint64_t cin = std::min<uint64_t>(cb, n_bytes ? n_bytes : 1);
  const uint64_t cout = compress_bound(cin, (uint32_t)std::min<uint64_t>(per, (cin + block_bytes - 1) / block_bytes));
  const bool pin_in = n_bytes && !is_pinned(h_in);
  const bool pin_out = is_pinned(h_out);
  int rc = hio_reserve(ctx, (cin + 255) & ~uint64_t(255), (cout + 255) & ~uint64_t(255), pin_in);
  if (rc) return rc;
  bzg_ctx::HostIo& h = ctx->hio;
  uint64_t pos = 0;
  int err = 0;
  // After chunk j's stream is done: its size, then its copy to the host.
  auto drain = [&](uint64_t j) -> int {
    const int b = (int)(j & 1);
    HIPX(hipEventSynchronize(h.comp_ev[b]));
    const uint64_t sz = h.hsize[b];
    if (err || pos + sz > out_cap) {
      err = BZG_ECAPACITY;
      return 0;
    }
    HIPX(hipStreamWaitEvent(h.down, h.comp_ev[b], 0));
    HIPX(hipMemcpyAsync(h_out + pos, h.dout[b], sz, hipMemcpyDeviceToHost, h.down));
    HIPX(hipEventRecord(h.out_ev[b], h.down));
    if (!pin_out) HIPX(hipEventSynchronize(h.out_ev[b]));
    pos += sz;
    return 0;
  };
  for (uint64_t i = 0; i < nc; i++) {
    const int b = (int)(i & 1);
    const uint64_t lo = i * cb, len = std::min<uint64_t>(cb, n_bytes - std::min(lo, n_bytes));
    // input: buffer b is free once chunk i - 2 has been compressed
    if (i >= 2) HIPX(hipStreamWaitEvent(h.up, h.comp_ev[b], 0));
    if (len) {
      const uint8_t* src = h_in + lo;
      if (pin_in) {  // staged: the pinned half is free once its last copy is done
        if (i >= 2) HIPX(hipEventSynchronize(h.in_ev[b]));
        memcpy(h.pin[b], src, len);
        src = h.pin[b];
      }
      HIPX(hipMemcpyAsync(h.din[b], src, len, hipMemcpyHostToDevice, h.up));
    }
    HIPX(hipEventRecord(h.in_ev[b], h.up));
    // compress chunk i into output buffer b (free once chunk i - 2's copy is done)
    HIPX(hipStreamWaitEvent(st, h.in_ev[b], 0));
    if (i >= 2) HIPX(hipStreamWaitEvent(st, h.out_ev[b], 0));
    std::vector<uint64_t> off;
    for (uint64_t o = 0; o < len; o += block_bytes) off.push_back(o);
    off.push_back(len);
    const uint32_t nblk = (uint32_t)off.size() - 1;
    rc = compress_common(ctx, h.din[b], nullptr, off.data(), nblk, nullptr, nullptr, 1, level, h.dout[b], nullptr,
                         nullptr, cout & ~uint64_t(3), h.dsize + b, nullptr, nullptr, 0, st);
    if (rc) {
      (void)hipStreamSynchronize(st);
      return rc;
    }
    HIPX(hipMemcpyAsync(h.hsize + b, h.dsize + b, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIPX(hipEventRecord(h.comp_ev[b], st));
    if (i >= 1 && (rc = drain(i - 1))) return rc;
  }
  if ((rc = drain(nc - 1))) return rc;
  HIPX(hipStreamSynchronize(h.down));
  HIPX(hipStreamSynchronize(st));
  if ((rc = status_result(ctx))) return rc;
  if (err) return fail(ctx, err, "output capacity too small for the streams");
  *h_out_bytes = pos;
  return 0;
}


}  // extern "C"

// ------------------------------------------------------------ decompression

namespace {

struct Stream {
  uint32_t b0, crc;
};

// The block layout of the input from its markers (bit position | end-marker
// flag << 63, the 32 bits after it | for end markers the 4 bytes where the
// next stream's header would start << 32): streams one after another, each
// "BZh" + level digit, blocks, end marker and CRC, padded to a byte.  Bytes
// after the last stream that do not start a stream header are ignored.
int lay_out_blocks(bzg_ctx* ctx, const std::vector<uint64_t>& cand, uint32_t first4, uint64_t n_bytes,
                   std::vector<DecBlk>& blocks, std::vector<Stream>& streams) {
  const size_t m = cand.size() / 2;
  uint64_t hb = 0;
  uint32_t hdr = first4;
  size_t i = 0;
  for (;;) {
    const uint32_t digit = hdr & 255u;
    if ((hdr >> 8) != 0x425A68u || digit < '1' || digit > '9') {
      if (streams.empty()) return fail(ctx, BZG_EDATA, "not a bzip2 stream (no BZh header)");
      break;
    }
    const uint32_t level = digit - '0';
    const uint64_t expect = hb * 8 + 32;
    if (i >= m || (cand[2 * i] & ~(1ull << 63)) != expect)
      return fail(ctx, BZG_EDATA, "no block or end marker right after the stream header at byte " + std::to_string(hb));
    Stream s{(uint32_t)blocks.size(), 0};
    for (;;) {
      if (i >= m) return fail(ctx, BZG_EDATA, "a stream without its end marker");
      const uint64_t pos = cand[2 * i] & ~(1ull << 63);
      const bool eos = cand[2 * i] >> 63;
      if (eos) {
        s.crc = (uint32_t)cand[2 * i + 1];
        hb = (pos + 80 + 7) / 8;
        hdr = (uint32_t)(cand[2 * i + 1] >> 32);
        i++;
        break;
      }
      if (i + 1 >= m) return fail(ctx, BZG_EDATA, "a block without a following marker");
      DecBlk d{};
      d.start = pos + 48;
      d.end = cand[2 * (i + 1)] & ~(1ull << 63);
      d.cap = 100000u * level;
      blocks.push_back(d);
      i++;
    }
    streams.push_back(s);
    if (hb + 4 > n_bytes) break;
    while (i < m && (cand[2 * i] & ~(1ull << 63)) < hb * 8 + 32) i++;  // (none expected)
  }
  return 0;
}

}  // namespace

extern "C" {

int decompress(bzg_ctx* ctx, const uint8_t* d_in, uint64_t n_bytes, uint8_t* d_out, uint64_t out_cap,
               uint64_t* d_out_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!d_out_bytes || !d_in || (out_cap && !d_out)) return fail(ctx, BZG_EINVAL, "null pointer");
  if (n_bytes < 14) return fail(ctx, BZG_EDATA, "input shorter than the smallest bzip2 stream");
  HIPX(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  // markers: counted per tile, then written in order; the host reads them back
  const uint64_t tiles = dec_find_tiles(n_bytes);
  if (tiles >= (1ull << 31)) return fail(ctx, BZG_EINVAL, "input too large");
  uint64_t count = 0;
  std::vector<uint64_t> cand;
  uint32_t first4 = 0;
  for (int round = 0; round < 2; round++) {
    Carve cv{nullptr};
    (void)cv.take<uint32_t>(tiles);
    (void)cv.take<uint64_t>(tiles + 1);
    (void)cv.take<uint64_t>(2 * count + 2);
    void* ws;
    int rc = get_ws(ctx, nullptr, 0, cv.used + 256, st, &ws);
    if (rc) return rc;
    Carve c2{(char*)ws};
    uint32_t* tile_cnt = c2.take<uint32_t>(tiles);
    uint64_t* tile_off = c2.take<uint64_t>(tiles + 1);
    uint64_t* dcand = c2.take<uint64_t>(2 * count + 2);
    HIPX(dec_find(d_in, n_bytes, 0, tile_cnt, nullptr, nullptr, 0, st));
    HIPX(dec_scan_counts(tile_cnt, (uint32_t)tiles, tile_off, st));
    if (round == 0) {
      HIPX(hipMemcpyAsync(&count, tile_off + tiles, sizeof(count), hipMemcpyDeviceToHost, st));
      HIPX(hipMemcpyAsync(&first4, d_in, 4, hipMemcpyDeviceToHost, st));
      if ((rc = end_ws(ctx, nullptr, st))) return rc;
      HIPX(hipStreamSynchronize(st));
      if (count == 0) return fail(ctx, BZG_EDATA, "no block or end marker found");
      if (count > (1ull << 26)) return fail(ctx, BZG_EDATA, "implausibly many markers");
      continue;
    }
    HIPX(dec_find(d_in, n_bytes, 1, tile_cnt, tile_off, dcand, count, st));
    cand.resize(2 * count);
    HIPX(hipMemcpyAsync(cand.data(), dcand, 16 * count, hipMemcpyDeviceToHost, st));
    if ((rc = end_ws(ctx, nullptr, st))) return rc;
    HIPX(hipStreamSynchronize(st));
  }
  first4 = __builtin_bswap32(first4);
  std::vector<DecBlk> blocks;
  std::vector<Stream> streams;
  int rc = lay_out_blocks(ctx, cand, first4, n_bytes, blocks, streams);
  if (rc) return rc;
  const uint32_t nb = (uint32_t)blocks.size(), ns = (uint32_t)streams.size();
  if (nb >= (1u << 24)) return fail(ctx, BZG_EINVAL, "too many blocks");
  // per block: BWT column, text and map ranges
  std::vector<uint32_t> sb0(ns + 1, 0), scrc(ns, 0);
  uint64_t lsum = 0;
  for (uint32_t b = 0; b < nb; b++) {
    blocks[b].l_off = lsum;
    lsum += blocks[b].cap;
  }
  for (uint32_t k = 0; k < ns; k++) {
    sb0[k] = streams[k].b0;
    scrc[k] = streams[k].crc;
  }
  sb0[ns] = nb;
  if (nb == 0) {  // empty streams only: their CRCs must be 0
    for (uint32_t k = 0; k < ns; k++)
      if (scrc[k]) return fail(ctx, BZG_EDATA, "an empty stream with a non-zero CRC");
    const uint64_t zero = 0;
    return upload(ctx, {{d_out_bytes, &zero, 8}}, st);
  }
  // the blocks by decreasing bit length, in classes decoded on streams of
  // their own: class k down to the longest block's bits >> DEC_CUT_SHIFT[k],
  // the last class the rest; the longer classes' serial Huffman decoding
  // then overlaps the shorter ones' later stages (batches of at least
  // DEC_SPLIT_MIN blocks)
  std::vector<uint32_t> order(nb);
  for (uint32_t b = 0; b < nb; b++) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
    return blocks[x].end - blocks[x].start > blocks[y].end - blocks[y].start;
  });
  struct Cls {
    uint32_t first, nb;
    uint64_t wt, rt, ct, ft;
  } cls[DEC_CLASSES] = {};
  uint32_t ncls = 0;
  {
    const uint64_t top = nb ? blocks[order[0]].end - blocks[order[0]].start : 0;
    uint32_t q = 0;
    for (uint32_t k = 0; k < DEC_CLASSES && q < nb; k++) {
      const uint32_t first = q;
      if (k + 1 == DEC_CLASSES || nb < DEC_SPLIT_MIN) {
        q = nb;
      } else {
        const uint64_t cut = top >> DEC_CUT_SHIFT[k];
        while (q < nb && blocks[order[q]].end - blocks[order[q]].start >= cut) q++;
      }
      if (q > first) cls[ncls++] = Cls{first, q - first, 0, 0, 0, 0};
    }
  }
  // per class: bounds on the work items the device plans from the decoded
  // lengths (walkers, run-length segments, move-to-front and FL chunks)
  uint64_t wt = 0, rt = 0, ct = 0, ft = 0;
  for (uint32_t k = 0; k < ncls; k++) {
    for (uint32_t q = cls[k].first; q < cls[k].first + cls[k].nb; q++) {
      const uint32_t cap = blocks[order[q]].cap;
      cls[k].wt += dec_walk_slots(cap);
      cls[k].rt += dec_rle_slots(cap);
      cls[k].ct += dec_mtf_chunks(cap);
      cls[k].ft += dec_fl_chunks(cap);
    }
    wt += cls[k].wt;
    rt += cls[k].rt;
    ct += cls[k].ct;
    ft += cls[k].ft;
  }
  const uint64_t tcap = out_cap / RLE_TILE + nb + 1;
  if (tcap >= (1ull << 31)) return fail(ctx, BZG_EINVAL, "out_cap too large");
  DecRun d{};
  auto carve = [&](char* base, DecRun& r, uint32_t** misc) -> size_t {
    Carve cv{base};
    r.blks = cv.take<DecBlk>(nb);
    r.order = cv.take<uint32_t>(nb);
    r.walk0 = cv.take<uint64_t>(nb + DEC_CLASSES);  // per class: its blocks + 1
    r.rle0 = cv.take<uint64_t>(nb + DEC_CLASSES);
    r.ch0 = cv.take<uint64_t>(nb + DEC_CLASSES);
    r.plan_cnt = cv.take<uint32_t>(nb);
    r.fl_off = cv.take<uint64_t>(nb + DEC_CLASSES);
    misc[0] = cv.take<uint32_t>(ns + 1);  // stream first blocks
    misc[1] = cv.take<uint32_t>(ns + 1);  // stream CRCs
    r.L = cv.take<uint8_t>(lsum + 64);
    r.T = cv.take<uint8_t>(lsum + 64);
    r.FL = cv.take<uint32_t>(lsum + 16);
    r.n_rows = cv.take<uint32_t>(nb);
    r.orig = cv.take<uint32_t>(nb);
    r.crc_want = cv.take<uint32_t>(nb);
    r.period = cv.take<uint32_t>(nb);
    r.out_len = cv.take<uint32_t>(nb);
    r.n_syms = cv.take<uint32_t>(nb);
    r.mtf0 = cv.take<uint8_t>((size_t)nb * 256);
    r.cs = cv.take<uint32_t>(ct);
    r.ce = cv.take<uint32_t>(ct);
    r.clen = cv.take<uint32_t>(ct);
    r.coff = cv.take<uint32_t>(ct);
    r.fl_cnt = cv.take<uint32_t>(ft * 256);
    r.fl_owner = cv.take<uint32_t>(ft);
    r.nxt = cv.take<uint32_t>(wt);
    r.steps = cv.take<uint32_t>(wt);
    r.pos = cv.take<uint32_t>(wt);
    r.summ = cv.take<uint64_t>(rt * 5);
    r.seg_in = cv.take<uint32_t>(rt);
    r.seg_off = cv.take<uint32_t>(rt);
    r.out_off = cv.take<uint64_t>(nb + 1);
    r.skip = cv.take<uint32_t>(4);
    misc[2] = cv.take<uint32_t>(nb + 1);      // CRC tiles: first tile per block
    misc[3] = cv.take<uint32_t>(PC_COUNT);    // tile count
    misc[4] = cv.take<uint32_t>(tcap + 1);    // tile -> block
    misc[5] = (uint32_t*)cv.take<char>(rle_tile_bytes() * (tcap + 1));
    misc[6] = cv.take<uint32_t>(tcap + 1);    // (run starts, unused here)
    misc[7] = cv.take<uint32_t>(tcap + 1);    // (RLE1 offsets, unused here)
    misc[8] = cv.take<uint32_t>(nb);          // (RLE1 lengths, unused here)
    misc[9] = cv.take<uint32_t>(nb);          // CRC of each decoded block
    return cv.used + 256;
  };
  uint32_t* misc[10];
  const size_t need = carve(nullptr, d, misc);
  void* ws;
  if ((rc = get_ws(ctx, nullptr, 0, need, st, &ws))) return rc;
  carve((char*)ws, d, misc);
  if ((rc = upload(ctx,
                   {{(void*)d.blks, blocks.data(), nb * sizeof(DecBlk)},
                    {(void*)d.order, order.data(), nb * 4},
                    {misc[0], sb0.data(), (ns + 1) * 4},
                    {misc[1], scrc.data(), ns * 4}},
                   st)))
    return rc;
  d.in = d_in;
  d.n_in = n_bytes;
  d.nb = nb;
  d.out = d_out;
  d.err = ctx->status;
  d.out_cap = out_cap;
  d.out_bytes = d_out_bytes;
  // the classes' runs: each its own range of every planned array
  DecRun dc[DEC_CLASSES];
  {
    uint32_t lo = 0;
    uint64_t w0 = 0, r0 = 0, c0 = 0, f0 = 0;
    for (uint32_t k = 0; k < ncls; k++) {
      DecRun& r = dc[k];
      r = d;
      r.nb = cls[k].nb;
      r.order = d.order + cls[k].first;
      r.plan_cnt = d.plan_cnt + cls[k].first;
      r.ch0 = d.ch0 + lo;  // offset arrays: nb + 1 entries per class
      r.fl_off = d.fl_off + lo;
      r.walk0 = d.walk0 + lo;
      r.rle0 = d.rle0 + lo;
      r.cs = d.cs + c0;
      r.ce = d.ce + c0;
      r.clen = d.clen + c0;
      r.coff = d.coff + c0;
      r.fl_cnt = d.fl_cnt + f0 * 256;
      r.fl_owner = d.fl_owner + f0;
      r.nxt = d.nxt + w0;
      r.steps = d.steps + w0;
      r.pos = d.pos + w0;
      r.summ = d.summ + r0 * 5;
      r.seg_in = d.seg_in + r0;
      r.seg_off = d.seg_off + r0;
      r.walk_total = cls[k].wt;
      r.rle_total = cls[k].rt;
      r.ch_total = cls[k].ct;
      r.fl_total = cls[k].ft;
      lo += cls[k].nb + 1;
      w0 += cls[k].wt;
      r0 += cls[k].rt;
      c0 += cls[k].ct;
      f0 += cls[k].ft;
    }
  }
  // the longer classes on the side streams (forked after this call's
  // uploads), the shortest on the call's stream, joined before the offsets
  if (ncls > 1 && !ctx->dec_fork) {
    for (hipStream_t& q : ctx->dec_side) HIPX(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    HIPX(hipEventCreateWithFlags(&ctx->dec_fork, hipEventDisableTiming));
    for (hipEvent_t& e : ctx->dec_join) HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (ncls > 1) HIPX(hipEventRecord(ctx->dec_fork, st));
  for (uint32_t k = 0; k + 1 < ncls; k++) {
    HIPX(hipStreamWaitEvent(ctx->dec_side[k], ctx->dec_fork, 0));
    HIPX(dec_run(dc[k], ctx->dec_side[k]));
    HIPX(hipEventRecord(ctx->dec_join[k], ctx->dec_side[k]));
  }
  HIPX(dec_run(dc[ncls - 1], st));
  for (uint32_t k = 0; k + 1 < ncls; k++) HIPX(hipStreamWaitEvent(st, ctx->dec_join[k], 0));
  HIPX(dec_offsets(d, nb, st));
  for (uint32_t k = 0; k < ncls; k++) HIPX(dec_output(dc[k], st));
  // block CRCs of the output (the compressor's tile CRC and its combination)
  HIPX(plan_slot_tiles(d.out_off, nb, misc[2], misc[3], st));
  {
    MapSet mm{};
    mm.map[0] = MapDesc{misc[2], misc[4], misc[3], (uint32_t)tcap, nb};
    mm.nmaps = 1;
    mm.err = ctx->status;
    HIPX(fill_maps(mm, st));
  }
  HIPX(rle1_tiles(d_out, persist_grid(tcap, ONE_TILE_EACH), misc[3], misc[4], misc[2], d.out_off, ctx->crc_tab,
                  ctx->crc_tab + CRC_POW_AT, misc[5], st));
  HIPX(rle1_blocks(nb, misc[2], d.out_off, ctx->crc_tab + CRC_POW_AT, misc[5], misc[6], misc[7], misc[8], misc[9], st));
  HIPX(dec_check(nb, misc[9], d.crc_want, ns, misc[0], misc[1], d.skip, ctx->status, st));
  return end_ws(ctx, nullptr, st);
}

}  // extern "C"

// ------------------------------------------------------------ field codecs

extern "C" {

uint64_t bzg_field_bound(int codec, uint64_t n_values) {
  if (codec < BZG_FIELD_NS32 || codec > BZG_FIELD_GFC64) return 0;
  return field_bound(codec, n_values);
}

int field_encode(bzg_ctx* ctx, int codec, const void* d_values, uint64_t n_values, uint8_t* d_out, uint64_t out_cap,
                 uint64_t* d_out_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (codec < BZG_FIELD_NS32 || codec > BZG_FIELD_GFC64) return fail(ctx, BZG_EINVAL, "unknown codec");
  if (!d_out || !d_out_bytes || (n_values && !d_values)) return fail(ctx, BZG_EINVAL, "null pointer");
  if (((uintptr_t)d_out & 7) || ((uintptr_t)d_values & (codec == BZG_FIELD_GFC64 ? 7 : 3)))
    return fail(ctx, BZG_EINVAL, "misaligned buffer");
  if (n_values >= (1ull << 34)) return fail(ctx, BZG_EINVAL, "too many values");
  if (out_cap < field_bound(codec, n_values))
    return fail(ctx, BZG_ECAPACITY, "out_cap below bzg_field_bound(): " + std::to_string(field_bound(codec, n_values)));
  HIPX(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nt = field_tiles(n_values);
  void* ws;
  int rc = get_ws(ctx, nullptr, 0, 16 * (nt + 1) + 512, st, &ws);
  if (rc) return rc;
  Carve cv{(char*)ws};
  uint64_t* tsum = cv.take<uint64_t>(nt + 1);
  uint64_t* toff = cv.take<uint64_t>(nt + 1);
  HIPX(field_encode_run(codec, d_values, n_values, d_out, d_out_bytes, tsum, toff, st));
  return end_ws(ctx, nullptr, st);
}

int field_decode(bzg_ctx* ctx, int codec, const uint8_t* d_in, uint64_t in_bytes, void* d_values, uint64_t n_values,
                 void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (codec < BZG_FIELD_NS32 || codec > BZG_FIELD_GFC64) return fail(ctx, BZG_EINVAL, "unknown codec");
  if (!d_in || (n_values && !d_values)) return fail(ctx, BZG_EINVAL, "null pointer");
  if (((uintptr_t)d_in & 7) || ((uintptr_t)d_values & (codec == BZG_FIELD_GFC64 ? 7 : 3)))
    return fail(ctx, BZG_EINVAL, "misaligned buffer");
  if (n_values >= (1ull << 34)) return fail(ctx, BZG_EINVAL, "too many values");
  // the fixed-size parts must be there: header, codes or index
  const uint64_t fixed = codec == BZG_FIELD_NS32 ? 8 + (n_values + 3) / 4
                         : codec == BZG_FIELD_GFC64 ? 8 + (n_values + 1) / 2
                                                    : 16 + 8 * ((n_values + 1023) / 1024);
  if (in_bytes < fixed) return fail(ctx, BZG_EDATA, "stream shorter than its fixed part");
  if (n_values == 0) return 0;
  HIPX(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nt = field_tiles(n_values);
  void* ws;
  int rc = get_ws(ctx, nullptr, 0, 32 * (nt + 1) + 1024, st, &ws);
  if (rc) return rc;
  Carve cv{(char*)ws};
  uint64_t* tsum = cv.take<uint64_t>(nt + 1);
  uint64_t* boff = cv.take<uint64_t>(nt + 1);
  uint64_t* rsum = cv.take<uint64_t>(nt + 1);
  uint64_t* roff = cv.take<uint64_t>(nt + 1);
  HIPX(field_decode_run(codec, d_in, in_bytes, n_values, d_values, tsum, boff, rsum, roff, ctx->status, st));
  return end_ws(ctx, nullptr, st);
}

}  // extern "C"

// ------------------------------------------------------------ tuning

extern "C" {

int bzg_set_tune(bzg_ctx* ctx, uint32_t mtf_chunk, uint32_t assign_groups, uint32_t count_steps) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  if ((mtf_chunk && mtf_chunk != 2048 && mtf_chunk != 4096) ||
      (assign_groups && assign_groups != 128 && assign_groups != 512) || count_steps > 1024)
    return fail(ctx, BZG_EINVAL, "mtf_chunk 0/2048/4096, assign_groups 0/128/512, count_steps 0..1024");
  ctx->tune.mtf_chunk = mtf_chunk;
  ctx->tune.assign_groups = assign_groups;
  ctx->tune.count_steps = count_steps;
  ctx->tune_set = mtf_chunk || assign_groups || count_steps;
  return 0;
}

int bzg_tune(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks, int level, void* stream,
             uint32_t* h_chosen) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!h_offsets || !n_blocks) return fail(ctx, BZG_EINVAL, "no blocks");
  int rc = check_compress(ctx, d_in, h_offsets, n_blocks, level);
  if (rc) return rc;
  HIPX(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const uint64_t total = h_offsets[n_blocks] - h_offsets[0];
  const uint64_t cap = (compress_bound(total, n_blocks) + 255) & ~uint64_t(255);
  uint8_t* out[2] = {nullptr, nullptr};
  uint64_t* nbytes = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (uint8_t* p : out)
      if (p) (void)hipFree(p);
    if (nbytes) (void)hipFree(nbytes);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc((void**)&out[0], cap) != hipSuccess || hipMalloc((void**)&out[1], cap) != hipSuccess ||
      hipMalloc((void**)&nbytes, 16) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(ctx, BZG_ENOMEM, "tuning buffers");
  }
  const Tune saved = ctx->tune;
  const bool saved_set = ctx->tune_set;
  std::vector<uint8_t> ref, got;
  uint64_t ref_n = 0;
  Tune best;
  double best_ms = 1e30;
  int points = 0;
  rc = 0;
  // every point must give the same bytes as the first (the built-in choices)
  for (uint32_t cs : {48u, 24u, 96u})
    for (uint32_t mc : {4096u, 2048u})
      for (uint32_t ag : {512u, 128u}) {
        if (rc) break;
        ctx->tune = Tune{mc, ag, cs};
        ctx->tune_set = true;
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && !rc; rep++) {
          (void)hipEventRecord(e0, st);
          rc = compress_common(ctx, d_in, nullptr, h_offsets, n_blocks, nullptr, nullptr, 1, level, out[points ? 1 : 0],
                               nullptr, nullptr, cap, nbytes + (points ? 1 : 0), nullptr, nullptr, 0, st);
          (void)hipEventRecord(e1, st);
          if (rc) break;
          if (hipEventSynchronize(e1) != hipSuccess) {
            rc = hip_fail(ctx, hipGetLastError(), "tune timing");
            break;
          }
          float t = 0;
          (void)hipEventElapsedTime(&t, e0, e1);
          ms = std::min(ms, t);
        }
        if (rc) break;
        if ((rc = status_result(ctx))) break;
        uint64_t n = 0;
        if (hipMemcpy(&n, nbytes + (points ? 1 : 0), 8, hipMemcpyDeviceToHost) != hipSuccess) {
          rc = hip_fail(ctx, hipGetLastError(), "tune read-back");
          break;
        }
        std::vector<uint8_t>& dst = points ? got : ref;
        dst.resize(n);
        if (n && hipMemcpy(dst.data(), out[points ? 1 : 0], n, hipMemcpyDeviceToHost) != hipSuccess) {
          rc = hip_fail(ctx, hipGetLastError(), "tune read-back");
          break;
        }
        if (points == 0) ref_n = n;
        if (points && (n != ref_n || memcmp(got.data(), ref.data(), n) != 0)) {
          rc = fail(ctx, BZG_EINTERNAL, "a tuning point changed the output bytes");
          break;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = ctx->tune;
        }
        points++;
      }
  ctx->tune = saved;
  ctx->tune_set = saved_set;
  cleanup();
  if (rc) return rc;
  const uint32_t bucket = tune_bucket(total, n_blocks);
  ctx->tune_table[bucket] = best;
  if (h_chosen) {
    h_chosen[0] = best.mtf_chunk;
    h_chosen[1] = best.assign_groups;
    h_chosen[2] = best.count_steps;
  }
  if (!ctx->tune_path.empty()) return save_tune_entry(ctx, bucket, best, best_ms);
  return 0;
}

}  // extern "C"

