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
// Single-pass exclusive scan in place, over a device-side element count
// (*count_ptr, at most cap, times mult), with decoupled look-back: a
// workgroup takes the next scan tile by ticket, publishes the tile's total,
// then its inclusive prefix once the tiles before it give theirs (wave 0
// reads 64 predecessors at a time and adds totals back to the nearest
// published prefix).  Tickets go out in dispatch order, so every tile waited
// on belongs to a running workgroup.  state[0] is the ticket counter and
// state[1 + t] tile t's word (flag << 62 | value); all must be zero at
// entry.  A wait that outlasts its bound sets ERR_BOUND and goes on (the
// result is then wrong but the kernel ends).
constexpr uint64_t LB_AGG = 1ull << 62, LB_PRE = 2ull << 62, LB_VAL = (1ull << 62) - 1;
constexpr uint32_t LB_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ void lb_publish(unsigned long long* p, uint64_t v) {
  __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_read(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_scan_lb(T* data, const uint32_t* __restrict__ count_ptr, uint32_t cap,
                                                uint32_t mult, unsigned long long* state, uint32_t* err) {
  __shared__ T sh[NT / BZG_WAVE + 1];
  __shared__ uint32_t s_tile;
  __shared__ T s_excl;
  const uint64_t n = (uint64_t)min(*count_ptr, cap) * mult;
  const uint64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd((unsigned int*)&state[0], 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    __syncthreads();
    if (t >= ntiles) break;
    const uint64_t base = (uint64_t)t * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) v[i] = data[min(base + i, n - 1)];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
      v[i] = base + i < n ? v[i] : T(0);
      acc += v[i];
    }
    T tot;
    const T ex = block_excl_sum<T, NT>(acc, sh, &tot);
    if (threadIdx.x < BZG_WAVE) {
      const uint32_t l = lane();
      if (l == 0) lb_publish(&state[1 + t], (t == 0 ? LB_PRE : LB_AGG) | (uint64_t)tot);
      uint64_t excl = 0;
      int64_t j = (int64_t)t - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        const int64_t idx = j - (int64_t)l;
        const uint64_t w = idx >= 0 ? lb_read(&state[1 + idx]) : LB_PRE;
        const uint64_t fl = w & ~LB_VAL;
        const uint64_t pm = __ballot(fl == LB_PRE), zm = __ballot(fl == 0);
        const uint32_t first_p = pm ? (uint32_t)(__ffsll((long long)pm) - 1) : 64u;
        const uint64_t need = first_p >= 63 ? ~0ull : ((2ull << first_p) - 1ull);
        if (zm & need) {
          if (++spins > LB_SPIN_LIMIT) {
            if (l == 0) atomicOr(err, ERR_BOUND);
            break;
          }
          __builtin_amdgcn_s_sleep(4);
          continue;
        }
        excl += wave_sum<uint64_t>(l <= first_p ? (w & LB_VAL) : 0ull);
        if (first_p < 64) break;
        j -= 64;
      }
      if (l == 0) {
        if (t) lb_publish(&state[1 + t], LB_PRE | ((excl + (uint64_t)tot) & LB_VAL));
        s_excl = (T)excl;
      }
    }
    __syncthreads();
    T run = s_excl + ex;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
      if (base + i < n) data[base + i] = run;
      run += v[i];
    }
  }
}

uint32_t scan_lb_states(uint64_t n) { return (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1); }

template <typename T>
static hipError_t scan_lb(T* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult, unsigned long long* state,
                          uint32_t* err, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_lb<T>, dim3(grid), dim3(NT), 0, s, data, count_ptr, cap, mult, state, err);
  return hipGetLastError();
}

hipError_t scan_lb_u32(uint32_t* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult,
                       unsigned long long* state, uint32_t* err, uint32_t grid, hipStream_t s) {
  return scan_lb<uint32_t>(data, count_ptr, cap, mult, state, err, grid, s);
}
hipError_t scan_lb_u64(uint64_t* data, const uint32_t* count_ptr, uint32_t cap, uint32_t mult,
                       unsigned long long* state, uint32_t* err, uint32_t grid, hipStream_t s) {
  return scan_lb<uint64_t>(data, count_ptr, cap, mult, state, err, grid, s);
}

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
