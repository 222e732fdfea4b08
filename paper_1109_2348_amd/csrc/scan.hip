// Device-wide exclusive prefix sum (reduce, scan of tile sums, downsweep).
// Sec. 2.1 of the paper singles the parallel prefix sum out as the primitive
// behind GPU run-length coding, lexicographic naming and variable-length
// packing; every later stage here uses it.
#include "common.hpp"
#include "internal.hpp"

namespace bzg {

constexpr int SCAN_ITEMS = 8;
constexpr size_t SCAN_TILE = size_t(NT) * SCAN_ITEMS;

template <typename T>
__global__ __launch_bounds__(NT) void k_scan_reduce(const T* __restrict__ in, size_t n, T* __restrict__ sums) {
  __shared__ T sh[NT / BZG_WAVE + 1];
  size_t base = (size_t)blockIdx.x * SCAN_TILE;
  T acc = 0;
  T x[SCAN_ITEMS];  // clamped loads, all in flight before any is added (n >= 1)
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) x[i] = in[min(base + (size_t)i * NT + threadIdx.x, n - 1)];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) acc += base + (size_t)i * NT + threadIdx.x < n ? x[i] : T(0);
  T tot = block_sum<T, NT>(acc, sh);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_scan_sums(T* sums, size_t ntiles) {
  __shared__ T sh[NT / BZG_WAVE + 1];
  T carry = 0;
  for (size_t b = 0; b < ntiles; b += NT) {
    size_t k = b + threadIdx.x;
    T v = sums[min(k, ntiles - 1)];  // clamped (ntiles >= 1)
    v = k < ntiles ? v : T(0);
    T tot;
    T ex = block_excl_sum<T, NT>(v, sh, &tot);
    if (k < ntiles) sums[k] = ex + carry;
    carry += tot;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_scan_down(const T* in, T* out, size_t n, const T* __restrict__ offs) {
  __shared__ T sh[NT / BZG_WAVE + 1];
  size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T acc = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) v[i] = in[min(base + i, n - 1)];  // clamped (n >= 1)
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    v[i] = base + i < n ? v[i] : T(0);
    acc += v[i];
  }
  T tot;
  T run = block_excl_sum<T, NT>(acc, sh, &tot) + offs[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    size_t k = base + i;
    if (k < n) out[k] = run;
    run += v[i];
  }
}

size_t scan_tmp_elems(size_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

// ----------------------------------------------------------------------------
// Exclusive scan in place over a device-side element count
// (min(*count_ptr, cap) * mult): per-tile sums, one workgroup scanning the
// sums, then every tile's local scan from its prefix.  Workgroups walk the
// tiles in a persistent loop, so a grid sized for the host bound works for
// any count.  sums: scan_lb_states(cap * mult) elements.
template <typename T>
__global__ __launch_bounds__(NT) void k_scan_reduce_dev(const T* __restrict__ in, const uint32_t* __restrict__ count_ptr,
                                                        uint32_t cap, uint32_t mult, T* __restrict__ sums) {
  __shared__ T sh[NT / BZG_WAVE + 1];
  const uint64_t n = (uint64_t)min(*count_ptr, cap) * mult;
  const uint32_t ntiles = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
  for (TileLoop it = tile_loop(ntiles); it.t < it.end; it.t += it.step) {
    const uint64_t base = (uint64_t)it.t * SCAN_TILE;
    T x[SCAN_ITEMS];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) x[i] = in[min(base + (uint64_t)i * NT + threadIdx.x, n - 1)];
    T acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) acc += base + (uint64_t)i * NT + threadIdx.x < n ? x[i] : T(0);
    const T tot = block_sum<T, NT>(acc, sh);
    if (threadIdx.x == 0) sums[it.t] = tot;
  }
}

constexpr int SUMS_NT = 1024;

template <typename T>
__global__ __launch_bounds__(SUMS_NT) void k_scan_sums_dev(T* sums, const uint32_t* __restrict__ count_ptr,
                                                           uint32_t cap, uint32_t mult) {
  __shared__ T sh[SUMS_NT / BZG_WAVE + 1];
  const uint64_t n = (uint64_t)min(*count_ptr, cap) * mult;
  const uint32_t ntiles = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
  T carry = 0;
  for (uint32_t b = 0; b < ntiles; b += SUMS_NT) {
    const uint32_t k = b + threadIdx.x;
    T v = sums[min(k, ntiles - 1)];  // clamped (ntiles >= 1 inside the loop)
    v = k < ntiles ? v : T(0);
    T tot;
    const T ex = block_excl_sum<T, SUMS_NT>(v, sh, &tot);
    if (k < ntiles) sums[k] = ex + carry;
    carry += tot;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_scan_down_dev(T* data, const uint32_t* __restrict__ count_ptr, uint32_t cap,
                                                      uint32_t mult, const T* __restrict__ sums) {
  __shared__ T sh[NT / BZG_WAVE + 1];
  constexpr int PV = 16 / sizeof(T);  // elements per 16-byte vector
  static_assert(SCAN_ITEMS % PV == 0, "whole vectors per thread");
  const uint64_t n = (uint64_t)min(*count_ptr, cap) * mult;
  const uint32_t ntiles = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
  const bool aligned = ((uintptr_t)data & 15u) == 0;
  for (TileLoop it = tile_loop(ntiles); it.t < it.end; it.t += it.step) {
    const uint64_t base = (uint64_t)it.t * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    // a thread's run of SCAN_ITEMS elements moves as whole 16-byte vectors
    // where it lies inside the count (every thread but the last one's)
    const bool whole = aligned && base + SCAN_ITEMS <= n;
    T v[SCAN_ITEMS];
    if (whole) {
#pragma unroll
      for (int j = 0; j < SCAN_ITEMS / PV; j++) {
        const uint4 q = *reinterpret_cast<const uint4*>(data + base + j * PV);
        __builtin_memcpy(&v[j * PV], &q, 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < SCAN_ITEMS; i++) v[i] = base + i < n ? data[base + i] : T(0);
    }
    T acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) acc += v[i];
    T tot;
    T run = block_excl_sum<T, NT>(acc, sh, &tot) + sums[it.t];
    T o[SCAN_ITEMS];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
      o[i] = run;
      run += v[i];
    }
    if (whole) {
#pragma unroll
      for (int j = 0; j < SCAN_ITEMS / PV; j++) {
        uint4 q;
        __builtin_memcpy(&q, &o[j * PV], 16);
        *reinterpret_cast<uint4*>(data + base + j * PV) = q;
      }
    } else {
#pragma unroll
      for (int i = 0; i < SCAN_ITEMS; i++)
        if (base + i < n) data[base + i] = o[i];
    }
    __syncthreads();
  }
}

uint32_t scan_lb_states(uint64_t n) { return (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1); }

template <typename T>
static hipError_t scan_dev(T* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult, T* sums, uint32_t grid,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_scan_reduce_dev<T>, dim3(grid), dim3(NT), 0, s, data, count_ptr, cap, mult, sums);
  hipLaunchKernelGGL(k_scan_sums_dev<T>, dim3(1), dim3(SUMS_NT), 0, s, sums, count_ptr, cap, mult);
  hipLaunchKernelGGL(k_scan_down_dev<T>, dim3(grid), dim3(NT), 0, s, data, count_ptr, cap, mult, (const T*)sums);
  return hipGetLastError();
}

hipError_t scan_lb_u32(uint32_t* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult,
                       unsigned long long* state, uint32_t* err, uint32_t grid, hipStream_t s) {
  (void)err;
  return scan_dev<uint32_t>(data, count_ptr, cap, mult, (uint32_t*)state, grid, s);
}
hipError_t scan_lb_u64(uint64_t* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult,
                       unsigned long long* state, uint32_t* err, uint32_t grid, hipStream_t s) {
  (void)err;
  return scan_dev<uint64_t>(data, count_ptr, cap, mult, (uint64_t*)state, grid, s);
}

// Tiles of a device-count scan over at most n elements (grid sizing).
uint32_t scan_dev_tiles(uint64_t n) { return (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE); }

}  // namespace bzg
