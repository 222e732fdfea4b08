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
// method must move, not what the hardware moved).  Collected after the call's
// final synchronisation.
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
  };
  std::vector<Pending> pending;
  std::map<std::string, ProfRec> acc;
  void collect();
};
extern thread_local Profiler* g_prof;

struct ProfScope {
  hipStream_t st;
  bool live = false;
  ProfScope(const char* name, hipStream_t s, double bytes);
  ~ProfScope();
};

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

// A run of equal-prefix rotations still to be ordered: SA rows
// [start, start+len) of block blk.  `base` is the segment's packed element
// offset (small segments) or first tile index (large segments).
struct SegRec {
  uint32_t start, len, blk, base;
};

// Device counters written by a sorting round and read back by the host.
// Counts appended to by every workgroup of a round, two per 64-bit word so
// that a workgroup takes its ranges with one atomic per word; the words sit
// on different cache lines.
struct RoundCounters {
  unsigned long long segs_small;  // segments for the next round | packed elements of small segments << 32
  uint32_t pad0[30];
  unsigned long long tiles_big;   // radix tiles of large segments | elements in large segments << 32
  uint32_t pad1[30];
  __host__ __device__ uint32_t n_segs() const { return (uint32_t)segs_small; }
  __host__ __device__ uint32_t small_total() const { return (uint32_t)(segs_small >> 32); }
  __host__ __device__ uint32_t big_tiles() const { return (uint32_t)tiles_big; }
  __host__ __device__ uint32_t big_active() const { return (uint32_t)(tiles_big >> 32); }
  __host__ __device__ uint32_t active() const { return small_total() + big_active(); }
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

// Device-wide exclusive scan; in == out allowed.  tmp needs scan_tmp_elems(n).
size_t scan_tmp_elems(size_t n);
hipError_t scan_excl_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, hipStream_t s);
hipError_t scan_excl_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp, hipStream_t s);

}  // namespace bzg
