// C ABI: argument checking, workspace planning and the launch sequence of
// every entry point declared in include/bzgpu.h.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bzgpu.h"
#include "internal.hpp"

namespace bzg {
// launchers from the kernel translation units
hipError_t rle1_tiles(const uint8_t*, uint32_t, const uint32_t*, const uint32_t*, const uint32_t*, const uint64_t*,
                      const uint32_t*, const uint32_t*, void*, hipStream_t);
hipError_t rle1_tile_copy(uint32_t, const uint32_t*, const void*, void*, hipStream_t);
hipError_t rle1_blocks(uint32_t, const uint32_t*, const uint64_t*, const uint32_t*, const void*, uint32_t*, uint32_t*,
                       uint32_t*, uint32_t*, hipStream_t);
hipError_t rle1_emit(const uint8_t*, uint32_t, const uint32_t*, const uint32_t*, const uint64_t*, const uint32_t*,
                     const uint32_t*, const uint64_t*, uint8_t*, hipStream_t);
hipError_t rle1_cut(const uint8_t*, uint32_t, const uint32_t*, const uint32_t*, const uint64_t*, const uint32_t*,
                    const uint32_t*, uint32_t, uint32_t*, hipStream_t);
size_t rle_tile_bytes();
size_t bwt_workspace_bytes(uint32_t N, uint32_t nb);
hipError_t bwt_sort(const uint8_t*, const std::vector<uint32_t>&, void*, size_t, RoundCounters*, Stager&,
                    uint32_t**, uint32_t**, int*, std::string&);
hipError_t bwt_output(const uint8_t*, const uint32_t*, uint32_t, uint32_t, const uint32_t*, uint8_t*, uint32_t*,
                      uint32_t*, hipStream_t);
size_t mtf_workspace_bytes(const std::vector<uint32_t>&);
hipError_t mtf_run(const uint8_t*, const uint32_t*, const std::vector<uint32_t>&, void*, size_t, uint16_t*,
                   const uint64_t*, uint32_t*, uint32_t*, uint32_t*, uint32_t*, Stager&, std::string&);
size_t block_tables_bytes();
hipError_t huff_run(uint32_t, const uint16_t*, const uint64_t*, const uint32_t*, uint32_t*, bool, const uint32_t*,
                    const uint64_t*, uint8_t*, uint8_t*, uint64_t*, void*, uint32_t*, uint32_t, const uint32_t*,
                    const uint32_t*, uint32_t, void*, hipStream_t);
size_t huff_workspace_bytes(uint32_t nb);
uint32_t huff_assign_groups(uint64_t ng);
hipError_t pack_layout(uint32_t, uint32_t, const uint32_t*, const uint64_t*, const void*, int, const uint64_t*,
                       uint64_t*, const uint32_t*, uint64_t*, hipStream_t);
hipError_t zero_streams(uint32_t, uint64_t, const uint64_t*, const uint64_t*, uint32_t*, hipStream_t);
hipError_t pack_run(uint32_t, const void*, int, const uint64_t*, const uint32_t*, const uint32_t*, const uint32_t*,
                    const uint64_t*, const uint8_t*, const uint8_t*, const uint64_t*, uint32_t, const uint32_t*,
                    const uint32_t*, const uint16_t*, const uint64_t*, const uint32_t*, int, uint32_t,
                    const uint64_t*, const uint64_t*, uint32_t*, hipStream_t);
hipError_t tables_export(uint32_t, const void*, uint8_t*, hipStream_t);
hipError_t body_sizes(uint32_t, const void*, const uint64_t*, uint64_t*, uint32_t*, hipStream_t);
}  // namespace bzg

namespace bzg {

thread_local Profiler* g_prof = nullptr;

ProfScope::ProfScope(const char* name, hipStream_t s, double bytes) : st(s) {
  if (g_prof && g_prof->on) {
    Profiler::Pending p{name, nullptr, nullptr, bytes};
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    (void)hipEventRecord(p.a, s);
    g_prof->pending.push_back(p);
    live = true;
  }
}

ProfScope::~ProfScope() {
  if (live) (void)hipEventRecord(g_prof->pending.back().b, st);
}

void Profiler::collect() {
  for (auto& p : pending) {
    float ms = 0;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ProfRec& r = acc[p.name];
      r.ms += ms;
      r.bytes += p.bytes;
      r.launches++;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  pending.clear();
}

}  // namespace bzg

using namespace bzg;

struct bzg_ctx {
  std::mutex mu;  // calls on one context run one at a time
  int device = 0;
  Profiler prof;
  std::string err;
  void* ws[2] = {nullptr, nullptr};
  size_t ws_cap[2] = {0, 0};
  void* pin = nullptr;
  size_t pin_cap = 0;
  void* stage = nullptr;  // pinned arena for uploads of host arrays
  size_t stage_cap = 0;
  // device: 4 x 256 byte-step tables (slicing by 4), 64 powers x^(8*2^j),
  // 256 tile shifts (mod P)
  uint32_t* crc_tab = nullptr;
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

#define HIPX(call)                                       \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// Scratch region `i` of at least `bytes`.  Growing waits for the device so
// no queued work still uses the old region.
int ensure_ws(bzg_ctx* ctx, int i, size_t bytes, void** out) {
  if (ctx->ws_cap[i] < bytes) {
    if (ctx->ws[i]) {
      HIPX(hipDeviceSynchronize());
      HIPX(hipFree(ctx->ws[i]));
      ctx->ws[i] = nullptr;
      ctx->ws_cap[i] = 0;
    }
    size_t want = bytes + bytes / 8 + (1 << 20);
    if (hipMalloc(&ctx->ws[i], want) != hipSuccess) {
      (void)hipGetLastError();
      ctx->ws[i] = nullptr;
      return fail(ctx, BZG_ENOMEM, "device scratch allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->ws_cap[i] = want;
  }
  *out = ctx->ws[i];
  return 0;
}

int ensure_pin(bzg_ctx* ctx, size_t bytes, void** out) {
  if (ctx->pin_cap < bytes) {
    if (ctx->pin) {
      HIPX(hipDeviceSynchronize());
      HIPX(hipHostFree(ctx->pin));
      ctx->pin = nullptr;
      ctx->pin_cap = 0;
    }
    size_t want = std::max(bytes, size_t(1) << 16);
    if (hipHostMalloc(&ctx->pin, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ctx->pin = nullptr;
      return fail(ctx, BZG_ENOMEM, "pinned host allocation failed");
    }
    ctx->pin_cap = want;
  }
  *out = ctx->pin;
  return 0;
}

// The upload arena, at least `bytes` large, bound to stream st.
int ensure_stage(bzg_ctx* ctx, size_t bytes, hipStream_t st, Stager* out) {
  if (ctx->stage_cap < bytes) {
    if (ctx->stage) {
      HIPX(hipDeviceSynchronize());
      HIPX(hipHostFree(ctx->stage));
      ctx->stage = nullptr;
      ctx->stage_cap = 0;
    }
    size_t want = std::max(bytes, size_t(1) << 20);
    if (hipHostMalloc(&ctx->stage, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ctx->stage = nullptr;
      return fail(ctx, BZG_ENOMEM, "pinned host allocation failed");
    }
    ctx->stage_cap = want;
  }
  out->base = (char*)ctx->stage;
  out->cap = ctx->stage_cap;
  out->used = ctx->stage_cap;  // full: the first upload drains the stream
  out->st = st;
  return 0;
}

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

struct Carve {
  char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t n) {
    size_t a = (used + 255) & ~size_t(255);
    used = a + n * sizeof(T);
    return reinterpret_cast<T*>(base + a);
  }
};

template <typename T>
size_t sz(size_t n) {
  return ((n * sizeof(T)) + 255) & ~size_t(255);
}

// Routes instrumented launches of one API call to the context's profiler.
struct ProfGuard {
  bzg_ctx* c;
  explicit ProfGuard(bzg_ctx* x) : c(x) { g_prof = &c->prof; }
  ~ProfGuard() {
    if (c->prof.on) c->prof.collect();
    g_prof = nullptr;
  }
};

// Tiles of `per` selector groups per block, from the per-block group
// capacities selb[b+1]-selb[b].
void group_tiles(const std::vector<uint64_t>& selb, uint32_t nb, uint32_t per, std::vector<uint32_t>& tile_blk,
                 std::vector<uint32_t>& blk_tile0) {
  tile_blk.clear();
  blk_tile0.assign(nb + 1, 0);
  for (uint32_t b = 0; b < nb; b++) {
    blk_tile0[b] = (uint32_t)tile_blk.size();
    uint64_t g = selb[b + 1] - selb[b];
    for (uint64_t q = 0; q < (g + per - 1) / per; q++) tile_blk.push_back(b);
  }
  blk_tile0[nb] = (uint32_t)tile_blk.size();
}

bool offsets_ok(const uint64_t* h, uint32_t nb) {
  for (uint32_t k = 0; k < nb; k++)
    if (h[k + 1] < h[k]) return false;
  return true;
}

}  // namespace

extern "C" {

int bzg_create(bzg_ctx** out, int hip_device) {
  if (!out) return BZG_EINVAL;
  *out = nullptr;
  bzg_ctx* ctx = new (std::nothrow) bzg_ctx();
  if (!ctx) return BZG_ENOMEM;
  ctx->device = hip_device;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = hipMalloc(&ctx->crc_tab, CRC_TAB_WORDS * sizeof(uint32_t));
  if (e == hipSuccess) {
    uint32_t h[CRC_TAB_WORDS];
    crc_tables(h, h + CRC_POW_AT);
    e = hipMemcpy(ctx->crc_tab, h, sizeof(h), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    delete ctx;
    return BZG_EHIP;
  }
  *out = ctx;
  return 0;
}

void bzg_destroy(bzg_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (int i = 0; i < 2; i++)
    if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  if (ctx->crc_tab) (void)hipFree(ctx->crc_tab);
  delete ctx;
}

const char* bzg_last_error(const bzg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int bzg_profile(bzg_ctx* ctx, int enable) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (enable) ctx->prof.acc.clear();
  ctx->prof.on = enable != 0;
  return 0;
}

int bzg_profile_read(bzg_ctx* ctx, char* buf, size_t cap) {
  if (!ctx || !buf || cap == 0) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
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

uint64_t bzg_compress_bound(uint64_t n_bytes, uint32_t n_blocks) {
  // every RLE1 byte becomes at most one 17-bit code (plus RUNA/RUNB digits,
  // which only replace zeros); generous per-block header allowance
  uint64_t rle = n_bytes + n_bytes / 4 + 4;
  uint64_t blocks = (uint64_t)n_blocks + rle / 100000 + 2;
  uint64_t bits = 32 + 80 + blocks * (105 + 16 + 256 + 18 + 6 * (5 + 258 * 33)) + rle * 17 + (rle / 50 + blocks) * 7;
  return ((bits + 7) / 8 + 3) & ~uint64_t(3);
}

int bwt_forward_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks,
                      uint8_t* d_bwt, uint32_t* d_primary, uint32_t* d_sa, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!h_offsets || !d_bwt || !d_primary || (n_blocks && !d_in)) return fail(ctx, BZG_EINVAL, "null pointer");
  if (n_blocks == 0) return 0;
  if (!offsets_ok(h_offsets, n_blocks)) return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (h_offsets[n_blocks] - h_offsets[0] >= (1ull << 32) - 4096) return fail(ctx, BZG_EINVAL, "batch too large");
  std::vector<uint32_t> off(n_blocks + 1);
  for (uint32_t k = 0; k <= n_blocks; k++) off[k] = (uint32_t)(h_offsets[k] - h_offsets[0]);
  for (uint32_t k = 0; k < n_blocks; k++) {
    uint32_t n = off[k + 1] - off[k];
    if (n == 0 || n > BZG_MAX_BLOCK) return fail(ctx, BZG_EINVAL, "block length outside 1..BZG_MAX_BLOCK");
  }
  hipStream_t st = (hipStream_t)stream;
  HIPX(hipSetDevice(ctx->device));
  const uint32_t N = off[n_blocks];
  void* ws;
  int rc = ensure_ws(ctx, 0, bwt_workspace_bytes(N, n_blocks), &ws);
  if (rc) return rc;
  void* pin;
  if ((rc = ensure_pin(ctx, 4096, &pin))) return rc;
  Stager stg;
  if ((rc = ensure_stage(ctx, 65536 + 8 * (size_t)n_blocks + N / 256, st, &stg))) return rc;
  const uint8_t* text = d_in + h_offsets[0];
  uint32_t *SA, *d_off;
  int rounds = 0;
  hipError_t e = bwt_sort(text, off, ws, ctx->ws_cap[0], (RoundCounters*)pin, stg, &SA, &d_off, &rounds, ctx->err);
  if (e != hipSuccess) return ctx->err.empty() ? hip_fail(ctx, e, "bwt_sort") : BZG_EHIP;
  HIPX(bwt_output(text, d_off, n_blocks, N, SA, d_bwt + h_offsets[0], d_primary, d_sa ? d_sa + h_offsets[0] : nullptr,
                  st));
  HIPX(hipStreamSynchronize(st));
  return 0;
}

int mtf_encode_batch(bzg_ctx* ctx, const uint8_t* d_bwt, const uint64_t* h_offsets, uint32_t n_blocks,
                     uint16_t* d_syms, uint32_t* d_nsyms, uint8_t* d_inuse, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!h_offsets || !d_syms || !d_nsyms || !d_inuse || (n_blocks && !d_bwt)) return fail(ctx, BZG_EINVAL, "null pointer");
  if (n_blocks == 0) return 0;
  if (!offsets_ok(h_offsets, n_blocks)) return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (((uintptr_t)d_inuse & 3) != 0) return fail(ctx, BZG_EINVAL, "d_inuse must be 4-byte aligned");
  if (h_offsets[n_blocks] - h_offsets[0] >= (1ull << 32) - 4096) return fail(ctx, BZG_EINVAL, "batch too large");
  std::vector<uint32_t> off(n_blocks + 1);
  for (uint32_t k = 0; k <= n_blocks; k++) off[k] = (uint32_t)(h_offsets[k] - h_offsets[0]);
  for (uint32_t k = 0; k < n_blocks; k++) {
    uint32_t n = off[k + 1] - off[k];
    if (n == 0 || n > BZG_MAX_BLOCK) return fail(ctx, BZG_EINVAL, "block length outside 1..BZG_MAX_BLOCK");
  }
  hipStream_t st = (hipStream_t)stream;
  HIPX(hipSetDevice(ctx->device));
  std::vector<uint64_t> sbase(n_blocks);
  for (uint32_t k = 0; k < n_blocks; k++) sbase[k] = h_offsets[k] + k;
  size_t need = sz<uint32_t>(n_blocks + 1) + sz<uint64_t>(n_blocks) + sz<uint32_t>((size_t)n_blocks * MAXA) +
                sz<uint32_t>(4) + mtf_workspace_bytes(off) + 4096;
  void* ws;
  int rc = ensure_ws(ctx, 1, need, &ws);
  if (rc) return rc;
  void* pin;
  if ((rc = ensure_pin(ctx, 4096, &pin))) return rc;
  Carve cv{(char*)ws};
  uint32_t* d_off = cv.take<uint32_t>(n_blocks + 1);
  uint64_t* d_sbase = cv.take<uint64_t>(n_blocks);
  uint32_t* d_freq = cv.take<uint32_t>((size_t)n_blocks * MAXA);
  uint32_t* d_err = cv.take<uint32_t>(4);
  void* rest = cv.take<char>(0);
  Stager stg;
  if ((rc = ensure_stage(ctx, 65536 + 16 * (size_t)n_blocks + off[n_blocks] / 256, st, &stg))) return rc;
  HIPX(stg.put_span({{d_off, off.data(), off.size() * 4}, {d_sbase, sbase.data(), sbase.size() * 8}}));
  hipError_t e = mtf_run(d_bwt + h_offsets[0], d_off, off, rest, ctx->ws_cap[1] - cv.used, d_syms, d_sbase, d_nsyms,
                         (uint32_t*)d_inuse, d_freq, d_err, stg, ctx->err);
  if (e != hipSuccess) return ctx->err.empty() ? hip_fail(ctx, e, "mtf") : BZG_EHIP;
  HIPX(hipMemcpyAsync(pin, d_err, 4, hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  if (*(uint32_t*)pin) return fail(ctx, BZG_EDATA, "mtf: symbol missing from the stack");
  return 0;
}

int huffman_encode_batch(bzg_ctx* ctx, const uint16_t* d_syms, const uint32_t* d_nsyms, const uint8_t* d_inuse,
                         const uint64_t* h_sym_offsets, uint32_t n_blocks, uint8_t* d_out,
                         const uint64_t* h_out_offsets, uint64_t* d_nbits, uint8_t* d_tables, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!h_sym_offsets || !h_out_offsets || !d_nbits || (n_blocks && (!d_syms || !d_nsyms || !d_inuse || !d_out)))
    return fail(ctx, BZG_EINVAL, "null pointer");
  if (n_blocks == 0) return 0;
  if (!offsets_ok(h_sym_offsets, n_blocks) || !offsets_ok(h_out_offsets, n_blocks))
    return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (((uintptr_t)d_out & 3) || (h_out_offsets[n_blocks] & 3) || (h_out_offsets[0] & 3) || ((uintptr_t)d_inuse & 3))
    return fail(ctx, BZG_EINVAL, "d_out/d_inuse must be 4-byte aligned and the output range multiples of 4");
  hipStream_t st = (hipStream_t)stream;
  HIPX(hipSetDevice(ctx->device));
  std::vector<uint64_t> sbase(n_blocks), selb(n_blocks + 1), obyte(n_blocks + 1);
  uint64_t ng = 0;
  for (uint32_t k = 0; k < n_blocks; k++) {
    sbase[k] = h_sym_offsets[k];
    selb[k] = ng;
    uint64_t cap = h_sym_offsets[k + 1] - h_sym_offsets[k];
    if (cap > 2ull * BZG_MAX_BLOCK + 2) return fail(ctx, BZG_EINVAL, "symbol capacity per block too large");
    ng += (cap + GROUP - 1) / GROUP;
  }
  selb[n_blocks] = ng;
  for (uint32_t k = 0; k <= n_blocks; k++) obyte[k] = h_out_offsets[k];
  std::vector<uint32_t> tile_blk, blk_tile0, atile_blk, ablk_tile0;
  group_tiles(selb, n_blocks, PACK_GROUPS, tile_blk, blk_tile0);
  const uint32_t atg = huff_assign_groups(ng);
  group_tiles(selb, n_blocks, atg, atile_blk, ablk_tile0);
  const uint32_t ntiles = (uint32_t)tile_blk.size(), natiles = (uint32_t)atile_blk.size();
  size_t need = sz<uint64_t>(n_blocks) * 2 + sz<uint64_t>(n_blocks + 1) * 2 + sz<uint32_t>((size_t)n_blocks * MAXA) +
                sz<uint8_t>(ng + 1) * 2 + sz<uint64_t>(ng + 1) * 2 + sz<uint64_t>(scan_tmp_elems(ng + 1)) +
                block_tables_bytes() * n_blocks + 256 + sz<uint32_t>(ntiles + 1) + sz<uint32_t>(natiles + 1) +
                2 * sz<uint32_t>(n_blocks + 1) + sz<uint64_t>(4) + sz<uint32_t>(4) + huff_workspace_bytes(n_blocks) +
                8192;
  void* ws;
  int rc = ensure_ws(ctx, 1, need, &ws);
  if (rc) return rc;
  void* pin;
  if ((rc = ensure_pin(ctx, 4096, &pin))) return rc;
  Carve cv{(char*)ws};
  uint64_t* d_sbase = cv.take<uint64_t>(n_blocks);
  uint64_t* d_selb = cv.take<uint64_t>(n_blocks + 1);
  uint64_t* d_obyte = cv.take<uint64_t>(n_blocks + 1);
  uint64_t* d_blkbit = cv.take<uint64_t>(n_blocks);
  uint32_t* d_freq = cv.take<uint32_t>((size_t)n_blocks * MAXA);
  uint8_t* d_sel = cv.take<uint8_t>(ng + 1);
  uint8_t* d_selmtf = cv.take<uint8_t>(ng + 1);
  uint64_t* d_gbits = cv.take<uint64_t>(ng + 1);
  uint64_t* d_gofs = cv.take<uint64_t>(ng + 1);
  uint64_t* d_stmp = cv.take<uint64_t>(scan_tmp_elems(ng + 1));
  void* d_tabs = cv.take<char>(block_tables_bytes() * n_blocks);
  uint32_t* d_tile_blk = cv.take<uint32_t>(ntiles + 1);
  uint32_t* d_blk_tile0 = cv.take<uint32_t>(n_blocks + 1);
  uint32_t* d_atile_blk = cv.take<uint32_t>(natiles + 1);
  uint32_t* d_ablk_tile0 = cv.take<uint32_t>(n_blocks + 1);
  uint64_t* d_info = cv.take<uint64_t>(4);
  uint32_t* d_err = cv.take<uint32_t>(4);
  void* d_hws = cv.take<char>(huff_workspace_bytes(n_blocks));
  Stager stg;
  if ((rc = ensure_stage(ctx, 65536 + 48 * (size_t)n_blocks + 4 * (size_t)(ntiles + natiles), st, &stg))) return rc;
  // (the first three, and the four tile maps, are adjacent in the carve)
  HIPX(stg.put_span({{d_sbase, sbase.data(), n_blocks * 8},
                     {d_selb, selb.data(), (n_blocks + 1) * 8},
                     {d_obyte, obyte.data(), (n_blocks + 1) * 8}}));
  HIPX(stg.put_span({{d_tile_blk, tile_blk.data(), ntiles * 4},
                     {d_blk_tile0, blk_tile0.data(), (n_blocks + 1) * 4},
                     {d_atile_blk, atile_blk.data(), natiles * 4},
                     {d_ablk_tile0, ablk_tile0.data(), (n_blocks + 1) * 4}}));
  HIPX(hipMemsetAsync(d_err, 0, 16, st));
  HIPX(huff_run(n_blocks, d_syms, d_sbase, d_nsyms, d_freq, true, (const uint32_t*)d_inuse, d_selb, d_sel, d_selmtf,
                d_gbits, d_tabs, d_err, natiles, d_atile_blk, d_ablk_tile0, atg, d_hws, st));
  HIPX(scan_excl_u64(d_gbits, d_gofs, ng + 1, d_stmp, st));
  HIPX(body_sizes(n_blocks, d_tabs, d_obyte, d_nbits, d_err, st));
  HIPX(pack_layout(n_blocks, 1, nullptr, nullptr, d_tabs, 1, d_obyte, d_blkbit, nullptr, d_info, st));
  HIPX(hipMemcpyAsync(pin, d_err, 4, hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  uint32_t ef = *(uint32_t*)pin;
  if (ef & 2u) return fail(ctx, BZG_EDATA, "huffman: symbol outside the alphabet");
  if (ef & 4u) return fail(ctx, BZG_ECAPACITY, "huffman: a block body does not fit its output range");
  HIPX(hipMemsetAsync(d_out + h_out_offsets[0], 0, h_out_offsets[n_blocks] - h_out_offsets[0], st));
  HIPX(pack_run(n_blocks, d_tabs, 1, d_blkbit, nullptr, nullptr, (const uint32_t*)d_inuse, d_selb, d_sel, d_selmtf,
                d_gofs, ntiles, d_tile_blk, d_blk_tile0, d_syms, d_sbase, d_nsyms, 9, 0, nullptr, d_info,
                (uint32_t*)d_out, st));
  if (d_tables) HIPX(tables_export(n_blocks, d_tabs, d_tables, st));
  HIPX(hipStreamSynchronize(st));
  return 0;
}

}  // extern "C"

namespace {

// One bzip2 stream per request: request r is input blocks
// [req_blocks[r], req_blocks[r+1]) and its stream goes to d_out + out_off[r],
// at most out_off[r+1] - out_off[r] bytes.  All requests' blocks go through
// every stage together.
int compress_impl(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks,
                  const uint32_t* req_blocks, uint32_t n_req, int level, uint8_t* d_out, const uint64_t* out_off,
                  uint64_t* h_out_bytes, uint32_t* h_n_blocks, hipStream_t st) {
  HIPX(hipSetDevice(ctx->device));
  const uint64_t in0 = n_blocks ? h_offsets[0] : 0;
  const uint64_t total = n_blocks ? h_offsets[n_blocks] - in0 : 0;
  if (total >= (1ull << 31)) return fail(ctx, BZG_EINVAL, "input too large for one call (2^31 bytes)");
  const uint8_t* in = d_in ? d_in + in0 : nullptr;
  // input blocks (relative to in), empty ones dropped; breq = owning request
  std::vector<uint64_t> boff{0};
  std::vector<uint32_t> breq;
  for (uint32_t r = 0; r < n_req; r++)
    for (uint32_t k = req_blocks[r]; k < req_blocks[r + 1]; k++)
      if (h_offsets[k + 1] > h_offsets[k]) {
        boff.push_back(h_offsets[k + 1] - in0);
        breq.push_back(r);
      }
  void* pin;
  int rc = ensure_pin(ctx, 64 * 1024 + 16 * (boff.size() + total / 100000 + 16) + 16 * (size_t)n_req, &pin);
  if (rc) return rc;
  Stager stg;
  if ((rc = ensure_stage(ctx, 65536 + 128 * boff.size() + total / 128 + 16 * (size_t)n_req, st, &stg))) return rc;
  uint32_t nb = (uint32_t)boff.size() - 1;
  if (h_n_blocks) *h_n_blocks = 0;
  if (nb == 0) {  // every stream is the 14-byte empty stream
    uint8_t* p = (uint8_t*)pin;
    const uint8_t empty[14] = {'B', 'Z', 'h', (uint8_t)('0' + level), 0x17, 0x72, 0x45, 0x38, 0x50, 0x90, 0, 0, 0, 0};
    memcpy(p, empty, 14);
    bool short_cap = false;
    for (uint32_t r = 0; r < n_req; r++) {
      h_out_bytes[r] = 14;
      short_cap |= out_off[r + 1] - out_off[r] < 14;
    }
    if (short_cap) return fail(ctx, BZG_ECAPACITY, "an empty stream needs 14 bytes");
    for (uint32_t r = 0; r < n_req; r++)
      HIPX(hipMemcpyAsync(d_out + out_off[r], p, 14, hipMemcpyHostToDevice, st));
    HIPX(hipStreamSynchronize(st));
    return 0;
  }
  const uint32_t limit = 100000u * (uint32_t)level;
  // ---- plan: RLE1 sizes, cutting blocks whose RLE1 output exceeds the limit
  const size_t max_nb = nb + total / 50000 + 4;
  const size_t max_tiles = total / RLE_TILE + 2 * max_nb + 4;
  size_t need1 = sz<uint64_t>(max_nb + 1) + sz<uint32_t>(max_tiles) + sz<uint32_t>(max_nb + 1) +
                 2 * (rle_tile_bytes() * max_tiles + 256) + sz<uint32_t>(max_tiles) * 4 + sz<uint32_t>(max_nb) * 4 +
                 sz<uint64_t>(max_nb + 1);
  void* ws1;
  if ((rc = ensure_ws(ctx, 1, need1, &ws1))) return rc;
  Carve c1{(char*)ws1};
  uint64_t* d_boff = c1.take<uint64_t>(max_nb + 1);
  uint32_t* d_tile_blk = c1.take<uint32_t>(max_tiles);
  uint32_t* d_blk_tile0 = c1.take<uint32_t>(max_nb + 1);
  void* d_rt[2] = {c1.take<char>(rle_tile_bytes() * max_tiles), c1.take<char>(rle_tile_bytes() * max_tiles)};
  uint32_t* d_tile_rs = c1.take<uint32_t>(max_tiles);
  uint32_t* d_tile_from = c1.take<uint32_t>(max_tiles);
  uint32_t* d_tile_ids = c1.take<uint32_t>(max_tiles);
  uint32_t* d_tile_out = c1.take<uint32_t>(max_tiles);
  uint32_t* d_rle_n = c1.take<uint32_t>(max_nb);
  uint32_t* d_crc = c1.take<uint32_t>(max_nb);
  uint32_t* d_cut_ids = c1.take<uint32_t>(max_nb);
  uint32_t* d_cuts = c1.take<uint32_t>(max_nb);
  uint64_t* d_rbase = c1.take<uint64_t>(max_nb + 1);
  std::vector<uint32_t> tile_blk, blk_tile0, rle_n;
  // after a cut, each block's origin: (block of the previous plan, offset of
  // its start in it); tiles that start at the same place and end at the same
  // place as before are copied, the others (a cut block's last tile and its
  // remainder) recomputed
  std::vector<uint32_t> org_blk, prev_tile0, tile_from, tile_ids;
  std::vector<uint64_t> org_delta, prev_boff;
  int cur = 0;  // tile-record buffer of the current plan
  uint32_t ntiles = 0;
  for (int iter = 0;; iter++) {
    nb = (uint32_t)boff.size() - 1;
    if (nb > max_nb) return fail(ctx, BZG_EINVAL, "internal: block plan overflow");
    tile_blk.clear();
    blk_tile0.assign(nb + 1, 0);
    for (uint32_t b = 0; b < nb; b++) {
      blk_tile0[b] = (uint32_t)tile_blk.size();
      uint64_t n = boff[b + 1] - boff[b];
      for (uint64_t t = 0; t < (n + RLE_TILE - 1) / RLE_TILE; t++) tile_blk.push_back(b);
    }
    blk_tile0[nb] = (uint32_t)tile_blk.size();
    ntiles = (uint32_t)tile_blk.size();
    HIPX(stg.put_span({{d_boff, boff.data(), (nb + 1) * 8},
                       {d_tile_blk, tile_blk.data(), ntiles * 4},
                       {d_blk_tile0, blk_tile0.data(), (nb + 1) * 4}}));
    if (iter == 0) {
      ProfScope ps("rle1_tiles", st, (double)(boff[nb] - boff[0]));
      HIPX(rle1_tiles(in, ntiles, nullptr, d_tile_blk, d_blk_tile0, d_boff, ctx->crc_tab, ctx->crc_tab + CRC_POW_AT,
                      d_rt[cur], st));
    } else {
      tile_from.assign(ntiles, ~0u);
      tile_ids.clear();
      double bytes = 0;
      for (uint32_t b = 0; b < nb; b++) {
        const uint32_t ob = org_blk[b];
        const uint64_t n = boff[b + 1] - boff[b], on = prev_boff[ob + 1] - prev_boff[ob];
        for (uint32_t t = blk_tile0[b]; t < blk_tile0[b + 1]; t++) {
          const uint64_t lo = (uint64_t)(t - blk_tile0[b]) * RLE_TILE;
          if (org_delta[b] == 0 && std::min<uint64_t>(lo + RLE_TILE, n) == std::min<uint64_t>(lo + RLE_TILE, on)) {
            tile_from[t] = prev_tile0[ob] + (t - blk_tile0[b]);
          } else {
            tile_ids.push_back(t);
            bytes += (double)(std::min<uint64_t>(lo + RLE_TILE, n) - lo);
          }
        }
      }
      const int nxt = cur ^ 1;
      HIPX(stg.put(d_tile_from, tile_from.data(), ntiles * 4));
      HIPX(rle1_tile_copy(ntiles, d_tile_from, d_rt[cur], d_rt[nxt], st));
      if (!tile_ids.empty()) {
        HIPX(stg.put(d_tile_ids, tile_ids.data(), tile_ids.size() * 4));
        ProfScope ps("rle1_tiles", st, bytes);
        HIPX(rle1_tiles(in, (uint32_t)tile_ids.size(), d_tile_ids, d_tile_blk, d_blk_tile0, d_boff, ctx->crc_tab,
                        ctx->crc_tab + CRC_POW_AT, d_rt[nxt], st));
      }
      cur = nxt;
    }
    HIPX(rle1_blocks(nb, d_blk_tile0, d_boff, ctx->crc_tab + CRC_POW_AT, d_rt[cur], d_tile_rs, d_tile_out, d_rle_n, d_crc,
                     st));
    uint32_t* h_rle = (uint32_t*)pin;
    HIPX(hipMemcpyAsync(h_rle, d_rle_n, nb * 4, hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    rle_n.assign(h_rle, h_rle + nb);
    std::vector<uint32_t> over;
    for (uint32_t b = 0; b < nb; b++)
      if (rle_n[b] > limit) over.push_back(b);
    if (over.empty()) break;
    if (iter > 64) return fail(ctx, BZG_EINVAL, "internal: block cutting did not converge");
    HIPX(stg.put(d_cut_ids, over.data(), over.size() * 4));
    HIPX(rle1_cut(in, (uint32_t)over.size(), d_cut_ids, d_blk_tile0, d_boff, d_tile_rs, d_tile_out, limit, d_cuts,
                  st));
    uint32_t* h_cut = (uint32_t*)pin;
    HIPX(hipMemcpyAsync(h_cut, d_cuts, over.size() * 4, hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    std::vector<uint64_t> nboff{0};
    std::vector<uint32_t> nbreq;
    org_blk.clear();
    org_delta.clear();
    size_t oi = 0;
    for (uint32_t b = 0; b < nb; b++) {
      uint64_t cut = 0;
      if (oi < over.size() && over[oi] == b) {
        cut = h_cut[oi++];
        if (cut == 0 || cut >= boff[b + 1] - boff[b]) return fail(ctx, BZG_EINVAL, "internal: bad block cut");
        nboff.push_back(boff[b] + cut);
        nbreq.push_back(breq[b]);
        org_blk.push_back(b);
        org_delta.push_back(0);
      }
      nboff.push_back(boff[b + 1]);
      nbreq.push_back(breq[b]);
      org_blk.push_back(b);
      org_delta.push_back(cut);
    }
    prev_boff.swap(boff);
    prev_tile0.swap(blk_tile0);
    boff.swap(nboff);
    breq.swap(nbreq);
  }
  // ---- streams: block range of every request (blocks are in request order)
  std::vector<uint32_t> rb(n_req + 1, nb);
  for (uint32_t b = nb; b-- > 0;) rb[breq[b]] = b;
  for (uint32_t r = n_req; r-- > 0;) rb[r] = std::min(rb[r], rb[r + 1]);
  // ---- RLE1 output layout
  std::vector<uint32_t> roff(nb + 1, 0);
  std::vector<uint64_t> rbase(nb + 1, 0);
  for (uint32_t b = 0; b < nb; b++) {
    roff[b + 1] = roff[b] + rle_n[b];
    rbase[b + 1] = roff[b + 1];
  }
  const uint32_t N = roff[nb];
  std::vector<uint64_t> sbase(nb), selb(nb + 1);
  uint64_t ng = 0;
  for (uint32_t b = 0; b < nb; b++) {
    sbase[b] = (uint64_t)roff[b] + b;
    selb[b] = ng;
    ng += ((uint64_t)rle_n[b] + 1 + GROUP - 1) / GROUP;
  }
  selb[nb] = ng;
  std::vector<uint32_t> ptile_blk, pblk_tile0, atile_blk, ablk_tile0;
  group_tiles(selb, nb, PACK_GROUPS, ptile_blk, pblk_tile0);
  const uint32_t atg = huff_assign_groups(ng);
  group_tiles(selb, nb, atg, atile_blk, ablk_tile0);
  const uint32_t nptiles = (uint32_t)ptile_blk.size(), natiles = (uint32_t)atile_blk.size();
  size_t bwt_ws = bwt_workspace_bytes(N, nb);
  size_t need0 = sz<uint8_t>(N + 64) * 2 + sz<uint32_t>(nb) + sz<uint16_t>((size_t)N + nb + 64) + sz<uint64_t>(nb) +
                 sz<uint32_t>(nb) + sz<uint32_t>((size_t)nb * 8) + sz<uint32_t>((size_t)nb * MAXA) + sz<uint32_t>(4) +
                 sz<uint64_t>(nb + 1) + sz<uint8_t>(ng + 1) * 2 + sz<uint64_t>(ng + 1) * 2 +
                 sz<uint64_t>(scan_tmp_elems(ng + 1)) + block_tables_bytes() * nb + 256 + sz<uint64_t>(nb) +
                 sz<uint32_t>(nptiles + 1) + sz<uint32_t>(nb + 1) + sz<uint64_t>(2 * (size_t)n_req + 2) +
                 sz<uint32_t>(n_req + 1) + sz<uint64_t>(n_req) + sz<uint32_t>(nb + 1) +
                 sz<uint32_t>(natiles + 1) + sz<uint32_t>(nb + 1) + huff_workspace_bytes(nb) +
                 std::max(bwt_ws, mtf_workspace_bytes(roff)) + 16384;
  void* ws0;
  if ((rc = ensure_ws(ctx, 0, need0, &ws0))) return rc;
  Carve c0{(char*)ws0};
  uint8_t* d_text = c0.take<uint8_t>(N + 64);
  uint8_t* d_L = c0.take<uint8_t>(N + 64);
  uint32_t* d_primary = c0.take<uint32_t>(nb);
  uint16_t* d_syms = c0.take<uint16_t>((size_t)N + nb + 64);
  // arrays uploaded together are carved next to each other (one copy each group)
  uint64_t* d_sbase = c0.take<uint64_t>(nb);
  uint32_t* d_roff = c0.take<uint32_t>(nb + 1);
  uint32_t* d_nsyms = c0.take<uint32_t>(nb);
  uint32_t* d_inuse = c0.take<uint32_t>((size_t)nb * 8);
  uint32_t* d_freq = c0.take<uint32_t>((size_t)nb * MAXA);
  uint32_t* d_err = c0.take<uint32_t>(4);
  uint64_t* d_selb = c0.take<uint64_t>(nb + 1);
  uint32_t* d_atile_blk = c0.take<uint32_t>(natiles + 1);
  uint32_t* d_ablk_tile0 = c0.take<uint32_t>(nb + 1);
  uint8_t* d_sel = c0.take<uint8_t>(ng + 1);
  uint8_t* d_selmtf = c0.take<uint8_t>(ng + 1);
  uint64_t* d_gbits = c0.take<uint64_t>(ng + 1);
  uint64_t* d_gofs = c0.take<uint64_t>(ng + 1);
  uint64_t* d_stmp = c0.take<uint64_t>(scan_tmp_elems(ng + 1));
  void* d_tabs = c0.take<char>(block_tables_bytes() * nb);
  uint64_t* d_blkbit = c0.take<uint64_t>(nb);
  uint32_t* d_ptile_blk = c0.take<uint32_t>(nptiles + 1);
  uint32_t* d_pblk_tile0 = c0.take<uint32_t>(nb + 1);
  uint64_t* d_info = c0.take<uint64_t>(2 * (size_t)n_req + 2);
  uint32_t* d_rb = c0.take<uint32_t>(n_req + 1);
  uint64_t* d_rout = c0.take<uint64_t>(n_req);
  void* d_hws = c0.take<char>(huff_workspace_bytes(nb));
  void* d_stage = c0.take<char>(0);
  size_t stage_bytes = ctx->ws_cap[0] - c0.used;
  HIPX(stg.put(d_rbase, rbase.data(), (nb + 1) * 8));
  {
    ProfScope ps("rle1_emit", st, (double)total + N);
    HIPX(rle1_emit(in, ntiles, d_tile_blk, d_blk_tile0, d_boff, d_tile_rs, d_tile_out, d_rbase, d_text, st));
  }
  // ---- BWT
  uint32_t *SA, *d_off;
  int rounds = 0;
  hipError_t e = bwt_sort(d_text, roff, d_stage, stage_bytes, (RoundCounters*)pin, stg, &SA, &d_off, &rounds, ctx->err);
  if (e != hipSuccess) return ctx->err.empty() ? hip_fail(ctx, e, "bwt_sort") : BZG_EHIP;
  HIPX(bwt_output(d_text, d_off, nb, N, SA, d_L, d_primary, nullptr, st));
  // ---- MTF + RUNA/RUNB (the sort's scratch is free again)
  HIPX(stg.put_span({{d_sbase, sbase.data(), nb * 8}, {d_roff, roff.data(), (nb + 1) * 4}}));
  e = mtf_run(d_L, d_roff, roff, d_stage, stage_bytes, d_syms, d_sbase, d_nsyms, d_inuse, d_freq, d_err, stg, ctx->err);
  if (e != hipSuccess) return ctx->err.empty() ? hip_fail(ctx, e, "mtf") : BZG_EHIP;
  // ---- Huffman tables, layout
  HIPX(stg.put_span({{d_selb, selb.data(), (nb + 1) * 8},
                     {d_atile_blk, atile_blk.data(), natiles * 4},
                     {d_ablk_tile0, ablk_tile0.data(), (nb + 1) * 4}}));
  HIPX(huff_run(nb, d_syms, d_sbase, d_nsyms, d_freq, false, d_inuse, d_selb, d_sel, d_selmtf, d_gbits, d_tabs, d_err,
                natiles, d_atile_blk, d_ablk_tile0, atg, d_hws, st));
  HIPX(scan_excl_u64(d_gbits, d_gofs, ng + 1, d_stmp, st));
  HIPX(stg.put_span({{d_rb, rb.data(), (n_req + 1) * 4}, {d_rout, out_off, n_req * 8}}));
  HIPX(pack_layout(nb, n_req, d_rb, d_rout, d_tabs, 0, nullptr, d_blkbit, d_crc, d_info, st));
  uint64_t* h_info = (uint64_t*)pin;
  HIPX(hipMemcpyAsync(h_info, d_info, 16 * (size_t)n_req, hipMemcpyDeviceToHost, st));
  HIPX(hipMemcpyAsync(h_info + 2 * (size_t)n_req, d_err, 4, hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  const uint32_t ef = (uint32_t)h_info[2 * (size_t)n_req];
  if (ef) return fail(ctx, BZG_EDATA, "internal: inconsistent symbol stream");
  uint64_t max_words = 0, out_total = 0;
  int short_r = -1;
  for (uint32_t r = 0; r < n_req; r++) {
    const uint64_t bits = h_info[2 * r], words = (bits + 31) / 32;
    h_out_bytes[r] = (bits + 7) / 8;
    out_total += h_out_bytes[r];
    max_words = std::max(max_words, words);
    if (words * 4 > out_off[r + 1] - out_off[r] && short_r < 0) short_r = (int)r;
  }
  if (h_n_blocks) *h_n_blocks = nb;
  if (short_r >= 0)
    return fail(ctx, BZG_ECAPACITY,
                "stream " + std::to_string(short_r) + " needs " +
                    std::to_string((h_info[2 * short_r] + 31) / 32 * 4) + " bytes (4-byte rounded)");
  // ---- pack
  HIPX(stg.put_span({{d_ptile_blk, ptile_blk.data(), nptiles * 4}, {d_pblk_tile0, pblk_tile0.data(), (nb + 1) * 4}}));
  {
    ProfScope ps("pack", st, 2.0 * N + (double)out_total);  // symbols in, streams out
    HIPX(zero_streams(n_req, max_words, d_rout, d_info, (uint32_t*)d_out, st));
    HIPX(pack_run(nb, d_tabs, 0, d_blkbit, d_crc, d_primary, d_inuse, d_selb, d_sel, d_selmtf, d_gofs, nptiles,
                  d_ptile_blk, d_pblk_tile0, d_syms, d_sbase, d_nsyms, level, n_req, d_rout, d_info,
                  (uint32_t*)d_out, st));
  }
  HIPX(hipStreamSynchronize(st));
  return 0;
}

}  // namespace

extern "C" {

int compress_blocks(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks, int level,
                    uint8_t* d_out, uint64_t out_cap, uint64_t* h_out_bytes, uint32_t* h_n_blocks, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!h_offsets || !d_out || !h_out_bytes) return fail(ctx, BZG_EINVAL, "null pointer");
  if (level < 1 || level > 9) return fail(ctx, BZG_EINVAL, "level must be 1..9");
  if (n_blocks && !offsets_ok(h_offsets, n_blocks)) return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (n_blocks && h_offsets[n_blocks] > h_offsets[0] && !d_in) return fail(ctx, BZG_EINVAL, "null input");
  if ((uintptr_t)d_out & 3) return fail(ctx, BZG_EINVAL, "d_out must be 4-byte aligned");
  const uint32_t rq[2] = {0, n_blocks};
  const uint64_t oo[2] = {0, out_cap & ~3ull};
  return compress_impl(ctx, d_in, h_offsets, n_blocks, rq, 1, level, d_out, oo, h_out_bytes, h_n_blocks,
                       (hipStream_t)stream);
}

int compress_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks,
                   const uint32_t* h_req_blocks, uint32_t n_req, int level, uint8_t* d_out,
                   const uint64_t* h_out_offsets, uint64_t* h_out_bytes, void* stream) {
  if (!ctx) return BZG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  ProfGuard pg(ctx);
  if (!h_offsets || !h_req_blocks || !h_out_offsets || !h_out_bytes || (n_req && !d_out))
    return fail(ctx, BZG_EINVAL, "null pointer");
  if (level < 1 || level > 9) return fail(ctx, BZG_EINVAL, "level must be 1..9");
  if (n_req > 65535) return fail(ctx, BZG_EINVAL, "at most 65535 requests per call");
  if (n_blocks && !offsets_ok(h_offsets, n_blocks)) return fail(ctx, BZG_EINVAL, "offsets decrease");
  if (n_blocks && h_offsets[n_blocks] > h_offsets[0] && !d_in) return fail(ctx, BZG_EINVAL, "null input");
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
  return compress_impl(ctx, d_in, h_offsets, n_blocks, h_req_blocks, n_req, level, d_out, h_out_offsets,
                       h_out_bytes, nullptr, (hipStream_t)stream);
}

}  // extern "C"
