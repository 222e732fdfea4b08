// Host-side declarations shared by the kernel translation units and the C
// ABI layer.  Not part of the public interface (that is include/bzgpu.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <initializer_list>
#include <map>
#include <string>
#include <vector>

namespace bzg {

// Optional per-kernel timing: HIP events recorded on the launch stream around
// each instrumented launch, with the launch's algorithmic bytes (the bytes the
// method must move, not what the hardware moved): a fixed part plus up to two
// device-side counts times a per-unit figure.  The counts are copied to a
// device buffer right after the launch (they may be reused later in the
// call) and read when the call's work is collected.
struct ProfRec {
  double ms = 0, bytes = 0;
  uint64_t launches = 0;
};
struct Profiler {
  bool on = false;
  struct Pending {
    const char* name;
    hipEvent_t a, b;
    double bytes;
    double per[2];
    int slot;  // first of two count slots, -1 = none
  };
  std::vector<Pending> pending;
  std::map<std::string, ProfRec> acc;
  uint32_t* slots = nullptr;  // device count snapshots
  int nslots = 0, used = 0;
  void collect();
};
extern thread_local Profiler* g_prof;

struct ProfScope {
  hipStream_t st;
  bool live = false;
  const uint32_t *c0 = nullptr, *c1 = nullptr;
  ProfScope(const char* name, hipStream_t s, double bytes, const uint32_t* count0 = nullptr, double per0 = 0,
            const uint32_t* count1 = nullptr, double per1 = 0);
  ~ProfScope();
};

// Launch parameters a context may set (bzg_set_tune, bzg_tune); every choice
// gives identical output.  0 = the built-in choice.  The API calls point
// g_tune at their context's values for the time they enqueue.
struct Tune {
  uint32_t mtf_chunk = 0;      // MTF rows per chunk: 2048 or 4096
  uint32_t assign_groups = 0;  // Huffman selector groups per assign tile: 128 or 512
  uint32_t count_steps = 0;    // small-segment sort: counting steps allowed per radix pass
};
extern thread_local const Tune* g_tune;

// Tuning constants (fixed; every choice gives identical output).
constexpr int NT = 256;                // threads per workgroup
constexpr uint32_t RADIX_TILE = 4096;  // elements per tile of a segment radix pass
constexpr uint32_t SMALL_T = 1024;     // packed elements per small-segment tile
constexpr uint32_t SMALL_MAX = 1024;   // segments up to this size are sorted in LDS
constexpr uint32_t SMALL_CAP = SMALL_T + SMALL_MAX;  // LDS capacity of a small tile
constexpr uint32_t RLE_TILE = 4096;    // input bytes per RLE1/CRC tile
constexpr uint32_t MTF_CHUNK = 4096;   // symbols per move-to-front chunk
constexpr uint32_t MAX_BLOCK = 1u << 21;  // largest block the sort accepts (ranks fit 21 bits)
constexpr int GROUP = 50;              // symbols per Huffman selector group
constexpr int MAXG = 6, MAXA = 258, MAXLEN = 17;
constexpr uint32_t CRC_POW_AT = 1024;                  // CRC table layout: 4 x 256 byte steps,
constexpr uint32_t CRC_TAB_WORDS = CRC_POW_AT + 64 + 256;  // then powers, then tile shifts
constexpr uint32_t PACK_GROUPS = 64;   // selector groups per bit-packing tile

// Per-block Huffman tables and sizes, written by the table kernels and read
// by the packing kernels.  G = 0 marks an empty block (no symbols).
struct BlockTables {
  uint32_t G, nsel, hdr_bits, alpha;
  uint64_t data_bits;
  uint8_t len[MAXG][MAXA];
  uint32_t code[MAXG][MAXA];
};

// Device-side error flags, OR-ed into the context's status word by the
// kernels of a call and reported (and cleared) by bzg_check.
constexpr uint32_t ERR_SYMBOL = 1u;    // a symbol outside its block's alphabet, or more symbols than slots
constexpr uint32_t ERR_CAPACITY = 2u;  // an output range too small: nothing was packed
constexpr uint32_t ERR_STREAM = 8u;    // a compressed stream that does not decode (corrupt or unsupported)
constexpr uint32_t ERR_BOUND = 4u;     // a device-side count exceeded its host bound (work was dropped)

// Persistent workgroup loops.  A kernel launched with G workgroups (a
// multiple of 8) walks tiles [0, n): the workgroups of XCD x = wg mod 8 take
// the x-th eighth of the range, each stepping by G / 8, so neighbouring tiles
// (the same block's rows, ranks and text) stay in that XCD's L2.  n may be a
// device-side count read by the kernel; G comes from the host's bound.
struct TileLoop {
  uint32_t t, end, step;
};
__device__ __forceinline__ TileLoop tile_loop(uint32_t n) {
  const uint32_t x = blockIdx.x & 7u, i = blockIdx.x >> 3, q = n >> 3, r = n & 7u;
  TileLoop L;
  const uint32_t lo = x * q + (x < r ? x : r);
  L.t = lo + i;
  L.end = lo + q + (x < r ? 1u : 0u);
  L.step = gridDim.x >> 3;
  return L;
}
// Workgroups for a launch over at most `bound` tiles: a multiple of 8, at
// most `cap`.  With cap >= bound every workgroup takes at most one tile (the
// hardware dispatches them as slots free up); a smaller cap makes the
// workgroups persistent.
inline uint32_t persist_grid(uint64_t bound, uint32_t cap) {
  uint64_t g = bound < cap ? bound : cap;
  g = (g + 7) & ~uint64_t(7);
  return (uint32_t)(g < 8 ? 8 : g);
}
constexpr uint32_t ONE_TILE_EACH = 0x7FFFFFF8u;  // cap for one tile per workgroup

// Workgroups of `kernel` (block of `threads`) that are resident on the
// device at once: the grid of a persistent launch whose tile count is
// usually far below its bound.
uint32_t resident_grid(const void* kernel, int threads);

// A run of equal-prefix rotations still to be ordered, too long for one
// small tile: SA rows [start, start+len) of block blk, radix tiles from
// `base` on.  (Small runs have no record: their first row is their mark in
// the block's packed head range.)
struct SegRec {
  uint32_t start, len, blk, base;
};

// Device counters written by a sorting round and read back by the host.
// Counts appended to by every workgroup of a round, two per 64-bit word so
// that a workgroup takes its ranges with one atomic per word; the words sit
// on different cache lines.
struct RoundCounters {
  unsigned long long segs_small;  // large segments for the next round | packed elements of small segments << 32
                                  // (the high word: the round's total, written by the round's first kernel)
  uint32_t pad0[30];
  unsigned long long tiles_big;   // radix tiles of large segments | elements in large segments << 32
  uint32_t pad1[30];
  __host__ __device__ uint32_t n_segs() const { return (uint32_t)segs_small; }
  __host__ __device__ uint32_t small_total() const { return (uint32_t)(segs_small >> 32); }
  __host__ __device__ uint32_t big_tiles() const { return (uint32_t)tiles_big; }
  __host__ __device__ uint32_t big_active() const { return (uint32_t)(tiles_big >> 32); }
  __host__ __device__ uint32_t active() const { return small_total() + big_active(); }
};

// The sort's workspace: SA rows, ranks, keys, radix buffers, histograms
// and scan state, segment lists, small-segment heads with their per-block
// counts and tile prefix, and three round-counter records, carved from one
// range by bwt_carve.
struct BwtSizes {
  size_t seg_cap, head_cap, owner_cap, hist_cap, state_cap;
};
struct BwtWork {
  uint32_t *SA, *rank, *key, *tmpK, *tmpV, *hist, *agg;
  unsigned long long* state;
  SegRec* segs[2];
  uint32_t* head[2];
  uint32_t* bcnt[2];   // per block: packed elements of its small segments
  uint32_t* tile_pre;  // per block: first small tile; [nslot] = all small tiles
  uint32_t* owner[2];
  RoundCounters* cnt;
  uint32_t nslot;
  BwtSizes z;
};
// Host bounds a sort is planned from: blocks (slots), rows, longest block,
// tiles of the first segments.
struct BwtBounds {
  uint32_t nslot, rows, max_len, init_tiles;
};

struct Bump {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  template <typename T>
  T* take(size_t n) {
    size_t a = (used + 255) & ~size_t(255);
    used = a + n * sizeof(T);
    return reinterpret_cast<T*>(base + a);
  }
};

// Uploads of host arrays through a pinned arena.  A copy from pageable host
// memory makes the host wait for the stream to reach it, which leaves the
// GPU idle while the host prepares the next launches; from pinned memory the
// copy stays asynchronous.  Each upload takes a fresh slice of the arena, so
// no queued copy sees its source overwritten; when the arena is full the
// stream is drained first and the arena reused.  It starts out full, so the
// first upload of a call also waits for work the stream still holds.
struct Stager {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  hipStream_t st = nullptr;
  hipError_t put(void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    if (bytes > cap) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    size_t at = (used + 255) & ~size_t(255);
    if (at > cap || cap - at < bytes) {
      const hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      at = 0;
    }
    memcpy(base + at, src, bytes);
    used = at + bytes;
    return hipMemcpyAsync(dst, base + at, bytes, hipMemcpyHostToDevice, st);
  }
  // Several arrays that lie in one device range, uploaded with one copy:
  // each source lands at its destination's offset in the range.  The bytes
  // between the arrays are overwritten too, so only alignment padding or
  // unused capacity of these same arrays may lie between them.
  struct Piece {
    void* dst;
    const void* src;
    size_t bytes;
  };
  hipError_t put_span(std::initializer_list<Piece> ps) {
    char *lo = nullptr, *hi = nullptr;
    for (const Piece& p : ps) {
      if (!p.bytes) continue;
      char* d = (char*)p.dst;
      if (!lo || d < lo) lo = d;
      if (!hi || d + p.bytes > hi) hi = d + p.bytes;
    }
    if (!lo) return hipSuccess;
    const size_t span = (size_t)(hi - lo);
    if (span > cap) {
      for (const Piece& p : ps) {
        const hipError_t e = put(p.dst, p.src, p.bytes);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
    size_t at = (used + 255) & ~size_t(255);
    if (at > cap || cap - at < span) {
      const hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      at = 0;
    }
    for (const Piece& p : ps)
      if (p.bytes) memcpy(base + at + ((char*)p.dst - lo), p.src, p.bytes);
    used = at + span;
    return hipMemcpyAsync(lo, base + at, span, hipMemcpyHostToDevice, st);
  }
};

// ---- launchers (defined in the kernel translation units) ----

// Arguments of the Huffman stage (huff.hip).
struct HuffArgs {
  uint32_t nb;  // blocks (slots)
  const uint16_t* syms;
  const uint64_t* sym_base;  // first symbol of each block in syms
  const uint32_t* nsyms;
  uint32_t* freq;  // nb * MAXA counts (input, or written when count_freq)
  const uint32_t* inuse;
  const uint64_t* sel_base;  // nb + 1 selector group bases
  uint8_t *sel, *selmtf;
  uint64_t* gbits;  // per-group data bits
  void* tabs;       // nb BlockTables
  uint32_t* err;
  const uint32_t *tile_blk, *blk_tile0, *n_tiles;  // assign tile map (device count)
  uint32_t tiles_cap, tile_groups;
  void* ws;  // huff_workspace_bytes(nb)
  const uint8_t* fixed = nullptr;  // precomputed tables (fixed_g x MAXA lengths) or null
  int fixed_g = 0;
  bool count_freq;           // symbols come from the caller: count and validate them
  const uint64_t* sym_off;   // (count_freq) nb + 1 symbol capacity offsets
  uint32_t* ns_eff;          // (count_freq) nb counts clamped to the capacities
};

// Decompression (decode.hip).  A block to decode, laid out by the host from
// the markers: its bits [start, end) after the block marker; `cap` (the
// stream's level limit) bytes of BWT column at l_off.
struct DecBlk {
  uint64_t start, end, l_off;
  uint32_t cap, pad;
};
// The arrays of one call, carved by the host.
// Decompression of a batch of at least DEC_SPLIT_MIN blocks decodes it in
// up to DEC_CLASSES classes of block length, each on a stream of its own.
constexpr uint32_t DEC_SPLIT_MIN = 64;
constexpr uint32_t DEC_CLASSES = 2;
constexpr int DEC_CUT_SHIFT[DEC_CLASSES - 1] = {2};  // class bounds: the longest block's bits >> these
struct DecRun {
  const uint8_t* in;
  uint64_t n_in;
  uint32_t nb;
  const DecBlk* blks;
  const uint32_t* order;  // the blocks decoded (global ids), by decreasing bit length
  uint8_t *L, *T, *out;
  uint32_t *n_rows, *orig, *crc_want, *err, *FL;
  uint32_t* n_syms;       // per block: Huffman symbols before end-of-block
  uint8_t* mtf0;          // per block: the 256-byte list move-to-front decoding starts from
  uint64_t* ch0;          // nb + 1 move-to-front chunk offsets (device-planned)
  uint64_t ch_total;      // move-to-front chunks at most (from the blocks' capacities)
  uint32_t *cs, *ce, *clen, *coff;  // per chunk slot: item range, output length and offset
  uint64_t fl_total;     // FL chunks at most (from the blocks' capacities)
  uint32_t* plan_cnt;    // per block: work items of the kind being planned
  uint64_t* fl_off;      // nb + 1 FL chunk offsets (device-planned)
  uint32_t* fl_cnt;      // 256 per FL chunk
  uint32_t* fl_owner;    // block of each FL chunk
  uint64_t* walk0;        // nb + 1 walker offsets (device-planned)
  uint64_t walk_total;    // walkers at most
  uint32_t *nxt, *steps, *pos, *period;
  uint64_t* rle0;         // nb + 1 segment offsets (device-planned)
  uint64_t rle_total;     // segments at most
  uint64_t* summ;  // 5 per segment slot
  uint32_t *seg_in, *seg_off, *out_len, *skip;
  uint64_t out_cap;
  uint64_t *out_off, *out_bytes;
};
hipError_t dec_find(const uint8_t* in, uint64_t n, int pass, uint32_t* tile_cnt, const uint64_t* tile_off,
                    uint64_t* cand, uint64_t cand_cap, hipStream_t st);
uint64_t dec_find_tiles(uint64_t n);
hipError_t dec_scan_counts(const uint32_t* cnt, uint32_t n, uint64_t* off, hipStream_t st);
uint32_t dec_walk_slots(uint32_t cap);
uint32_t dec_rle_slots(uint32_t cap);
uint32_t dec_mtf_chunks(uint32_t cap);
uint32_t dec_fl_chunks(uint32_t cap);
// A class of blocks (d.order, d.nb of them) decoded through the run-length
// chain; then the offsets of every block; then each class's output.
hipError_t dec_run(const DecRun& d, hipStream_t st);
hipError_t dec_offsets(const DecRun& d, uint32_t nb, hipStream_t st);
hipError_t dec_output(const DecRun& d, hipStream_t st);
hipError_t dec_check(uint32_t nb, const uint32_t* crc_got, const uint32_t* crc_want, uint32_t n_streams,
                     const uint32_t* stream_b0, const uint32_t* stream_crc, const uint32_t* skip, uint32_t* err,
                     hipStream_t st);

// Field codecs (fields.hip); codec ids as in the public header.
uint64_t field_bound(int codec, uint64_t n);
uint64_t field_tiles(uint64_t n);
hipError_t field_encode_run(int codec, const void* vals, uint64_t n, uint8_t* out, uint64_t* out_bytes,
                            uint64_t* tile_sum, uint64_t* tile_off, hipStream_t st);
hipError_t field_decode_run(int codec, const uint8_t* z, uint64_t in_bytes, uint64_t n, void* vals, uint64_t* tile_sum,
                            uint64_t* byte_off, uint64_t* res_sum, uint64_t* res_off, uint32_t* err, hipStream_t st);

size_t bwt_workspace_bytes(uint32_t N, uint32_t nb);
bool bwt_carve(void* ws, size_t ws_bytes, uint32_t N, uint32_t nb, BwtWork& w);
int bwt_rounds(uint32_t max_len);
void bwt_warm_grids();  // computes the sort's resident grid sizes once
hipError_t bwt_sort(BwtWork& w, const uint8_t* text, const uint32_t* d_off, const uint32_t* init_tiles,
                    const BwtBounds& bd, uint32_t* err, int* rounds, hipStream_t st);
hipError_t bwt_output(const uint8_t* text, const uint32_t* d_off, uint32_t nb, const uint32_t* n_rows, uint32_t cap,
                      const uint32_t* SA, uint8_t* L, uint32_t* primary, uint32_t* sa_local, hipStream_t st);

// Device-wide exclusive scan; in == out allowed.  tmp needs scan_tmp_elems(n).
size_t scan_tmp_elems(size_t n);
hipError_t scan_excl_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, hipStream_t s);
hipError_t scan_excl_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp, hipStream_t s);
// Exclusive scan in place over min(*count_ptr, cap) * mult elements (a
// device count): three launches (tile sums, their scan, the tiles' scans).
// state: scan_lb_states(cap * mult) elements of scratch; grid: workgroups of
// the tile passes (they loop over the tiles).
uint32_t scan_lb_states(uint64_t n);
uint32_t scan_dev_tiles(uint64_t n);
hipError_t scan_lb_u32(uint32_t* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult,
                       unsigned long long* state, uint32_t* err, uint32_t grid, hipStream_t s);
hipError_t scan_lb_u64(uint64_t* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult,
                       unsigned long long* state, uint32_t* err, uint32_t grid, hipStream_t s);

}  // namespace bzg
