// Wave64 / workgroup primitives shared by the CDNA4 kernels.
//
// Everything here is written for 64-lane wavefronts: ballots are 64-bit
// masks, the in-wave rank of a lane among lanes holding the same digit is
// popcount(peers & lanemask_lt), and workgroup scans combine per-wave totals
// through LDS.  The prefix sum (Sec. 2.1 of the paper: the primitive behind
// run-length coding, naming and variable-length packing) is the workhorse.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BZG_WAVE 64

namespace bzg {

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane()) - 1ull; }

template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
#pragma unroll
  for (int d = 1; d < BZG_WAVE; d <<= 1) {
    T u = __shfl_up(v, d, BZG_WAVE);
    if ((int)lane() >= d) v += u;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_max(T v) {
#pragma unroll
  for (int d = 1; d < BZG_WAVE; d <<= 1) {
    T u = __shfl_up(v, d, BZG_WAVE);
    if ((int)lane() >= d) v = u > v ? u : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, BZG_WAVE);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    T u = __shfl_xor(v, d, BZG_WAVE);
    v = u > v ? u : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v ^= __shfl_xor(v, d, BZG_WAVE);
  return v;
}

// Exclusive sum over a workgroup of NT threads.  `sh` needs NT/64 + 1 slots.
// Every thread must call it.  Returns the exclusive prefix; *total gets the sum.
template <typename T, int NT>
__device__ __forceinline__ T block_excl_sum(T v, T* sh, T* total) {
  constexpr int NW = NT / BZG_WAVE;
  T inc = wave_incl_sum(v);
  const int w = threadIdx.x / BZG_WAVE;
  if (lane() == BZG_WAVE - 1) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int i = 0; i < NW; i++) {
      T t = sh[i];
      sh[i] = acc;
      acc += t;
    }
    sh[NW] = acc;
  }
  __syncthreads();
  T r = inc - v + sh[w];
  *total = sh[NW];
  __syncthreads();
  return r;
}

// Inclusive max over a workgroup (values must be >= `lo`).
template <typename T, int NT>
__device__ __forceinline__ T block_incl_max(T v, T* sh, T lo) {
  constexpr int NW = NT / BZG_WAVE;
  T inc = wave_incl_max(v);
  const int w = threadIdx.x / BZG_WAVE;
  if (lane() == BZG_WAVE - 1) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = lo;
    for (int i = 0; i < NW; i++) {
      T t = sh[i];
      sh[i] = acc;
      acc = t > acc ? t : acc;
    }
    sh[NW] = acc;
  }
  __syncthreads();
  T c = sh[w];
  T r = c > inc ? c : inc;
  __syncthreads();
  return r;
}

template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  T tot;
  (void)block_excl_sum<T, NT>(v, sh, &tot);
  return tot;
}

// Lanes of the wave holding the same 8-bit digit (restricted to `valid`).
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t valid) {
  uint64_t m = valid;
#pragma unroll
  for (int b = 0; b < 8; b++) {
    uint64_t bal = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return m;
}

// Copies n elements from global memory to LDS with NTH threads: BATCH loads
// per thread in flight at a time (clamped indices, so no load sits under a
// branch and waits alone).
template <int NTH, int BATCH, typename T>
__device__ __forceinline__ void stage_to_lds(T* dst, const T* __restrict__ src, uint32_t n) {
  for (uint32_t base = 0; base < n; base += NTH * BATCH) {
    T v[BATCH];
#pragma unroll
    for (int j = 0; j < BATCH; j++) v[j] = src[min(base + j * NTH + threadIdx.x, n - 1u)];
#pragma unroll
    for (int j = 0; j < BATCH; j++) {
      const uint32_t i = base + j * NTH + threadIdx.x;
      if (i < n) dst[i] = v[j];
    }
  }
}

// Up to 16 bytes starting at p (1 <= n <= 16 of them valid) as 4 little-endian
// words: byte i of the span is byte i%4 of word i/4.  Reads the aligned
// dwords that hold at least one valid byte (so never a page the span does not
// touch) and realigns them with v_alignbyte; bytes past n are unspecified.
__device__ __forceinline__ void load16(const uint8_t* p, uint32_t n, uint32_t out[4]) {
  const uintptr_t a = (uintptr_t)p;
  // global address space: a pointer rebuilt from an integer would otherwise
  // be loaded through flat instructions, which also hold up LDS waits
  typedef const uint32_t __attribute__((address_space(1)))* gword;
  const gword w = (gword)(a & ~(uintptr_t)3);
  const uint32_t sh = (uint32_t)(a & 3u);
  const uint32_t nd = (sh + n + 3u) >> 2;  // dwords holding valid bytes (<= 5)
  uint32_t v[5];
#pragma unroll
  for (int j = 0; j < 5; j++) v[j] = (uint32_t)j < nd ? w[j] : 0u;
#pragma unroll
  for (int j = 0; j < 4; j++) out[j] = __builtin_amdgcn_alignbyte(v[j + 1], v[j], sh);
}

// Workgroups are dispatched to the 8 XCDs round-robin by workgroup id.  This
// maps workgroup id -> logical tile so that every XCD runs one contiguous
// range of tiles: neighbouring tiles (the same block's rows, ranks and text)
// then share that XCD's L2.  A bijection on [0, n).
constexpr uint32_t NXCD = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t wg, uint32_t n) {
  const uint32_t x = wg % NXCD, i = wg / NXCD, q = n / NXCD, r = n % NXCD;
  return x * q + (x < r ? x : r) + i;
}

// ---------------------------------------------------------------- CRC-32
// The bzip2 block CRC is non-reflected (MSB first) with polynomial
// 0x04C11DB7; in GF(2)[x] the register after data B (from zero) is
// B(x) * x^32 mod P, and the register over A||B is reg(A) * x^(8|B|) xor
// reg(B).  Chunks are therefore CRC'd independently and combined by
// multiplying with powers of x.
constexpr uint32_t CRC_POLY = 0x04C11DB7u;

__device__ __forceinline__ uint32_t gf2_mulmod(uint32_t a, uint32_t b) {
  uint32_t r = 0;
  for (int i = 31; i >= 0; i--) {
    r = (r << 1) ^ ((r & 0x80000000u) ? CRC_POLY : 0u);
    if ((b >> i) & 1u) r ^= a;
  }
  return r;
}

// x^(8 * nbytes) mod P from a table pw[j] = x^(8 * 2^j) mod P.
__device__ __forceinline__ uint32_t gf2_xpow8(uint64_t nbytes, const uint32_t* pw) {
  uint32_t r = 1u;  // the polynomial 1
  int j = 0;
  while (nbytes) {
    if (nbytes & 1ull) r = gf2_mulmod(r, pw[j]);
    nbytes >>= 1;
    j++;
  }
  return r;
}

}  // namespace bzg
