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

template <typename T>
static hipError_t scan_excl(const T* in, T* out, size_t n, T* tmp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nt), dim3(NT), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(NT), 0, s, tmp, nt);
  hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)nt), dim3(NT), 0, s, in, out, n, (const T*)tmp);
  return hipGetLastError();
}

hipError_t scan_excl_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, hipStream_t s) {
  return scan_excl<uint32_t>(in, out, n, tmp, s);
}
hipError_t scan_excl_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp, hipStream_t s) {
  return scan_excl<uint64_t>(in, out, n, tmp, s);
}

}  // namespace bzg
