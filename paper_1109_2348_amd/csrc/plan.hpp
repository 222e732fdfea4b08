// Device-side planning records shared by the planning kernels (plan.hip) and
// the C ABI layer.  Internal; not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace bzg {

// Indices into the device count record written by k_plan_layout.
enum PlanCount : int {
  PC_ROWS = 0,         // total length of all slots (RLE1 bytes / BWT rows / MTF rows)
  PC_SORT_TILES = 1,   // RADIX_TILE tiles of the sort's first segments
  PC_CHUNKS = 2,       // MTF chunks
  PC_ASSIGN_TILES = 3, // Huffman assign tiles
  PC_PACK_TILES = 4,   // bit-packing tiles
  PC_GROUPS_LO = 5,    // selector groups (64-bit, low and high words)
  PC_GROUPS_HI = 6,
  PC_RLE_TILES = 7,    // RLE1 tiles over the slots
  PC_IN_TILES = 8,     // RLE1 tiles over the input blocks (block cutting)
  PC_COUNT = 16
};

struct PlanArgs {
  uint32_t nslot;
  uint32_t mtf_chunk;      // MTF chunk rows (when chunk0 is wanted)
  uint32_t assign_groups;  // groups per Huffman assign tile
  int groups_plus_one;     // groups = ceil((len + 1) / 50) (room for EOB) or ceil(len / 50)
};

struct PlanOut {  // every pointer optional
  uint32_t* roff;        // nslot + 1 exclusive offsets of the lengths
  uint64_t* sbase;       // nslot: roff + slot (symbol bases)
  uint64_t* selb;        // nslot + 1 selector group bases
  uint32_t* sort_tile0;  // nslot + 1
  SegRec* segs0;         // nslot first segments (needs roff and sort_tile0)
  uint32_t* chunk0;      // nslot + 1
  uint32_t* asg_tile0;   // nslot + 1
  uint32_t* pack_tile0;  // nslot + 1
  uint32_t* cnt;         // PC_COUNT counts
};

struct MapDesc {
  const uint32_t* tile0;  // nslot + 1 first tiles
  uint32_t* owner;        // tile -> slot
  const uint32_t* total;  // device-side tile count
  uint32_t bound;         // host bound on the tile count (owner capacity)
  uint32_t nslot;
};
struct MapSet {
  MapDesc map[5];
  int nmaps;
  uint32_t* err;
};

// Pieces an input block of n bytes can be cut into at limit L (RLE1 bytes):
// a piece that is not the last holds at least L - 1 RLE1 bytes (one more
// input byte adds at most 2) and so at least ceil(4 (L - 1) / 5) input bytes
// (RLE1 expands by at most 5/4).
__host__ __device__ inline uint32_t max_pieces(uint64_t n, uint32_t L) {
  if (n == 0) return 0;
  if (n + n / 4 <= L) return 1;
  const uint64_t min_in = (4ull * (L - 1) + 4) / 5;
  return (uint32_t)(n / min_in + 1);
}

hipError_t plan_input(const uint64_t* in_off, uint32_t n_in, uint32_t L, uint32_t* slot_base, uint32_t* tile0,
                      uint32_t* cnt, uint64_t* in_rel, hipStream_t st);
hipError_t call_init(uint32_t* skip, uint32_t* rb, uint32_t nb, uint64_t* rout, uint64_t cap, hipStream_t st);
hipError_t plan_slot_tiles(const uint64_t* slot_in, uint32_t nslot, uint32_t* tile0, uint32_t* cnt, hipStream_t st);
hipError_t plan_layout(const uint32_t* len32, const uint64_t* off64, const PlanArgs& a, const PlanOut& o,
                       hipStream_t st);
hipError_t fill_maps(const MapSet& m, hipStream_t st);
hipError_t fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);

}  // namespace bzg
