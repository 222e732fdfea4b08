// Device-side planning.  Every size a call depends on -- block offsets after
// RLE1, tile and chunk maps, selector group bases -- is computed here from
// device arrays, so a call enqueues its kernels without reading anything back
// (the paper's Sec. 4 point: data stays on the device).  The host only knows
// upper bounds (from the caller's block offsets) and sizes grids and
// workspace from them.
//
// Blocks are "slots": an input block whose RLE1 output may exceed the
// decoder's limit owns as many slots as pieces it can be cut into; slots a
// block does not need stay empty and are skipped by every stage.
#include "common.hpp"
#include "internal.hpp"
#include "plan.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

namespace bzg {

constexpr int PNT = 1024;  // threads of the single-workgroup planning scans

// Exclusive scan over n values, one workgroup of PNT threads, each thread
// taking a contiguous run of the values.  `get(i)` gives value i; `put(i, ex)`
// receives the exclusive prefix of i (i == n gets the total).
template <typename T, typename Get, typename Put>
__device__ void wg_scan(uint32_t n, Get get, Put put, T* sh) {
  const uint32_t per = (n + PNT - 1) / PNT;
  const uint32_t i0 = min(threadIdx.x * per, n), i1 = min(i0 + per, n);
  T s = 0;
  for (uint32_t i = i0; i < i1; i++) s += get(i);
  T tot;
  T run = block_excl_sum<T, PNT>(s, sh, &tot);
  for (uint32_t i = i0; i < i1; i++) {
    const T v = get(i);
    put(i, run);
    run += v;
  }
  if (threadIdx.x == 0) put(n, tot);
}

__device__ __forceinline__ uint32_t ceil_div(uint64_t a, uint32_t b) { return (uint32_t)((a + b - 1) / b); }

// Input blocks -> slots.  in_off: the caller's n_in + 1 offsets (absolute;
// in0 = in_off[0] is subtracted).  Writes in_rel (the offsets relative to
// in0), slot_base[k] (exclusive scan of the block's slot count, n_in + 1
// entries) and, per block that may need cutting, its tile range over
// RLE_TILE-byte tiles (tile0[k], total in cnt[0]; other blocks get none).
__global__ __launch_bounds__(PNT) void k_plan_input(const uint64_t* __restrict__ in_off, uint32_t n_in, uint32_t L,
                                                    uint32_t* __restrict__ slot_base, uint32_t* __restrict__ tile0,
                                                    uint32_t* __restrict__ cnt, uint64_t* __restrict__ in_rel) {
  __shared__ uint32_t sh[PNT / BZG_WAVE + 1];
  const uint64_t in0 = in_off[0];
  auto len = [&](uint32_t k) { return in_off[k + 1] - in_off[k]; };
  wg_scan<uint32_t>(
      n_in, [&](uint32_t k) { return max_pieces(len(k), L); },
      [&](uint32_t k, uint32_t ex) { slot_base[k] = ex; }, sh);
  __syncthreads();
  // only blocks that may need cutting are measured whole (the others fit)
  wg_scan<uint32_t>(
      n_in, [&](uint32_t k) { return max_pieces(len(k), L) > 1 ? ceil_div(len(k), RLE_TILE) : 0u; },
      [&](uint32_t k, uint32_t ex) {
        tile0[k] = ex;
        if (k == n_in) cnt[0] = ex;
      },
      sh);
  for (uint32_t k = threadIdx.x; k <= n_in; k += PNT) in_rel[k] = in_off[k] - in0;
}

// Per-call device scalars: the skip flag cleared, and (when given) a
// one-request range table {0, nb} / {0, cap}.
__global__ void k_call_init(uint32_t* __restrict__ skip, uint32_t* __restrict__ rb, uint32_t nb,
                            uint64_t* __restrict__ rout, uint64_t cap) {
  if (threadIdx.x == 0) {
    *skip = 0;
    if (rb) {
      rb[0] = 0;
      rb[1] = nb;
    }
    if (rout) {
      rout[0] = 0;
      rout[1] = cap;
    }
  }
}

// Slots -> RLE1 tiles: tile0[s] over the slots' input ranges slot_in, total
// in cnt[0].
__global__ __launch_bounds__(PNT) void k_plan_slot_tiles(const uint64_t* __restrict__ slot_in, uint32_t nslot,
                                                         uint32_t* __restrict__ tile0, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t sh[PNT / BZG_WAVE + 1];
  wg_scan<uint32_t>(
      nslot, [&](uint32_t s) { return ceil_div(slot_in[s + 1] - slot_in[s], RLE_TILE); },
      [&](uint32_t s, uint32_t ex) {
        tile0[s] = ex;
        if (s == nslot) cnt[0] = ex;
      },
      sh);
}

// The layout of every stage after RLE1, from the slots' lengths (RLE1 output
// lengths, or the differences of 64-bit offsets): RLE1 offsets, symbol
// bases (block k's symbols at offset_k + k), selector group bases, and the
// tile maps' first tiles.  One workgroup; totals in p->cnt.
__global__ __launch_bounds__(PNT) void k_plan_layout(const uint32_t* __restrict__ len32,
                                                     const uint64_t* __restrict__ off64, PlanArgs a, PlanOut o) {
  __shared__ uint32_t sh[PNT / BZG_WAVE + 1];
  __shared__ uint64_t sh64[PNT / BZG_WAVE + 1];
  const uint32_t n = a.nslot;
  auto len = [&](uint32_t s) -> uint32_t { return len32 ? len32[s] : (uint32_t)(off64[s + 1] - off64[s]); };
  auto groups = [&](uint32_t s) -> uint32_t {
    const uint32_t l = len(s);
    return l == 0 ? 0u : ceil_div((uint64_t)l + (a.groups_plus_one ? 1u : 0u), GROUP);
  };
  if (o.roff)
    wg_scan<uint32_t>(
        n, [&](uint32_t s) { return len(s); },
        [&](uint32_t s, uint32_t ex) {
          o.roff[s] = ex;
          if (o.sbase && s < n) o.sbase[s] = (uint64_t)ex + s;
          if (s == n) o.cnt[PC_ROWS] = ex;
        },
        sh);
  __syncthreads();
  if (o.sort_tile0)
    wg_scan<uint32_t>(
        n, [&](uint32_t s) { return ceil_div(len(s), RADIX_TILE); },
        [&](uint32_t s, uint32_t ex) {
          o.sort_tile0[s] = ex;
          if (s == n) o.cnt[PC_SORT_TILES] = ex;
        },
        sh);
  __syncthreads();
  if (o.chunk0)
    wg_scan<uint32_t>(
        n, [&](uint32_t s) { return ceil_div(len(s), a.mtf_chunk); },
        [&](uint32_t s, uint32_t ex) {
          o.chunk0[s] = ex;
          if (s == n) o.cnt[PC_CHUNKS] = ex;
        },
        sh);
  __syncthreads();
  if (o.selb)
    wg_scan<uint64_t>(
        n, [&](uint32_t s) { return (uint64_t)groups(s); },
        [&](uint32_t s, uint64_t ex) {
          o.selb[s] = ex;
          if (s == n) {
            o.cnt[PC_GROUPS_LO] = (uint32_t)ex;
            o.cnt[PC_GROUPS_HI] = (uint32_t)(ex >> 32);
          }
        },
        sh64);
  __syncthreads();
  if (o.asg_tile0)
    wg_scan<uint32_t>(
        n, [&](uint32_t s) { return ceil_div(groups(s), a.assign_groups); },
        [&](uint32_t s, uint32_t ex) {
          o.asg_tile0[s] = ex;
          if (s == n) o.cnt[PC_ASSIGN_TILES] = ex;
        },
        sh);
  __syncthreads();
  if (o.pack_tile0)
    wg_scan<uint32_t>(
        n, [&](uint32_t s) { return ceil_div(groups(s), PACK_GROUPS); },
        [&](uint32_t s, uint32_t ex) {
          o.pack_tile0[s] = ex;
          if (s == n) o.cnt[PC_PACK_TILES] = ex;
        },
        sh);
  __syncthreads();
  // the sort's first segments: one per non-empty slot (its whole block)
  if (o.segs0)
    for (uint32_t s = threadIdx.x; s < n; s += PNT) {
      SegRec r;
      r.start = o.roff[s];
      r.len = len(s);
      r.blk = s;
      r.base = o.sort_tile0[s];
      o.segs0[s] = r;
    }
}

// Owner of every tile of up to four maps: owner[t] = the last slot s with
// tile0[s] <= t (empty slots share their tile0 with the next slot, so the
// last one is the slot that holds tile t).  Grid-stride over the maps'
// bounds; tiles at or past a map's device-side total are left alone.
__global__ __launch_bounds__(NT) void k_fill_maps(MapSet m) {
  const uint64_t stride = (uint64_t)gridDim.x * NT;
  for (int q = 0; q < m.nmaps; q++) {
    const MapDesc d = m.map[q];
    const uint32_t total = *d.total;
    if (total > d.bound) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(m.err, ERR_BOUND);
    }
    const uint32_t n = min(total, d.bound);
    for (uint64_t t = (uint64_t)blockIdx.x * NT + threadIdx.x; t < n; t += stride) {
      uint32_t lo = 0, hi = d.nslot - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (d.tile0[mid] <= (uint32_t)t) lo = mid; else hi = mid - 1;
      }
      d.owner[t] = lo;
    }
  }
}

// A fill kernel (memset equivalent that stays valid inside captured graphs).
__global__ __launch_bounds__(NT) void k_fill32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * NT) p[i] = v;
}

hipError_t plan_input(const uint64_t* in_off, uint32_t n_in, uint32_t L, uint32_t* slot_base, uint32_t* tile0,
                      uint32_t* cnt, uint64_t* in_rel, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_input, dim3(1), dim3(PNT), 0, st, in_off, n_in, L, slot_base, tile0, cnt, in_rel);
  return hipGetLastError();
}

hipError_t call_init(uint32_t* skip, uint32_t* rb, uint32_t nb, uint64_t* rout, uint64_t cap, hipStream_t st) {
  hipLaunchKernelGGL(k_call_init, dim3(1), dim3(64), 0, st, skip, rb, nb, rout, cap);
  return hipGetLastError();
}

hipError_t plan_slot_tiles(const uint64_t* slot_in, uint32_t nslot, uint32_t* tile0, uint32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_slot_tiles, dim3(1), dim3(PNT), 0, st, slot_in, nslot, tile0, cnt);
  return hipGetLastError();
}

hipError_t plan_layout(const uint32_t* len32, const uint64_t* off64, const PlanArgs& a, const PlanOut& o,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_plan_layout, dim3(1), dim3(PNT), 0, st, len32, off64, a, o);
  return hipGetLastError();
}

hipError_t fill_maps(const MapSet& m, hipStream_t st) {
  uint64_t tot = 0;
  for (int q = 0; q < m.nmaps; q++) tot += m.map[q].bound;
  const uint32_t g = (uint32_t)std::min<uint64_t>((tot + NT - 1) / NT + 1, 4096);
  if (m.nmaps) hipLaunchKernelGGL(k_fill_maps, dim3(g), dim3(NT), 0, st, m);
  return hipGetLastError();
}

uint32_t resident_grid(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, uint32_t> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({dev, kernel});
  if (it != cache.end()) return it->second;
  int occ = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess || occ < 1) occ = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  const uint32_t g = persist_grid((uint64_t)occ * cus, ONE_TILE_EACH);
  cache[{dev, kernel}] = g;
  return g;
}

hipError_t fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint32_t g = (uint32_t)std::min<uint64_t>((n + NT - 1) / NT, 2048);
  hipLaunchKernelGGL(k_fill32, dim3(g), dim3(NT), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace bzg
