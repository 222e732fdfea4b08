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

#include <limits>

#define BZG_WAVE 64

namespace bzg {

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane()) - 1ull; }

// DPP lane moves (GFX9 controls): row_shr:n (0x110 + n) gives lane l of each
// 16-lane row the value of lane l - n of the same row; row_bcast:15 (0x142)
// gives a row lane 15 of the row before; row_bcast:31 (0x143) gives lane 31;
// wave_shr:1 (0x138) gives lane l the value of lane l - 1.  ROW_MASK picks the
// rows written.  Lanes not written, or without a source lane, get `idle`.
// These move data through the VALU, with none of the LDS round trip of a
// ds_bpermute shuffle.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t idle, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)idle, (int)v, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_move(T idle, T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(
        T, dpp32<CTRL, ROW_MASK>(__builtin_bit_cast(uint32_t, idle), __builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t i = __builtin_bit_cast(uint64_t, idle), x = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = dpp32<CTRL, ROW_MASK>((uint32_t)i, (uint32_t)x);
    const uint32_t hi = dpp32<CTRL, ROW_MASK>((uint32_t)(i >> 32), (uint32_t)(x >> 32));
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// The value of lane 63, in every lane.
template <typename T>
__device__ __forceinline__ T wave_last(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), BZG_WAVE - 1));
  } else {
    const uint64_t x = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, BZG_WAVE - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), BZG_WAVE - 1);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// Inclusive scan over the wave for an associative op with identity `id`:
// steps of 1, 2, 4, 8 lanes inside each 16-lane row, then each row takes the
// total of the rows before it (row 1 from row 0 and row 3 from row 2, then
// rows 2 and 3 from lane 31).
template <typename T, typename Op>
__device__ __forceinline__ T wave_incl_scan(T v, T id, Op op) {
  v = op(v, dpp_move<0x111, 0xF>(id, v));
  v = op(v, dpp_move<0x112, 0xF>(id, v));
  v = op(v, dpp_move<0x114, 0xF>(id, v));
  v = op(v, dpp_move<0x118, 0xF>(id, v));
  v = op(v, dpp_move<0x142, 0xA>(id, v));
  v = op(v, dpp_move<0x143, 0xC>(id, v));
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
  return wave_incl_scan(v, T(0), [](T a, T b) { return a + b; });
}

template <typename T>
__device__ __forceinline__ T wave_incl_max(T v) {
  return wave_incl_scan(v, std::numeric_limits<T>::lowest(), [](T a, T b) { return a > b ? a : b; });
}

__device__ __forceinline__ uint64_t wave_incl_or(uint64_t v) {
  return wave_incl_scan(v, uint64_t(0), [](uint64_t a, uint64_t b) { return a | b; });
}

// Lane l gets lane l - 1's value; lane 0 gets `first`.
template <typename T>
__device__ __forceinline__ T wave_shr1(T first, T v) {
  return dpp_move<0x138, 0xF>(first, v);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  return wave_last(wave_incl_sum(v));
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  return wave_last(wave_incl_max(v));
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  return wave_last(wave_incl_scan(v, 0u, [](uint32_t a, uint32_t b) { return a | b; }));
}

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
  return wave_last(wave_incl_scan(v, 0u, [](uint32_t a, uint32_t b) { return a ^ b; }));
}

// Exclusive sum over a workgroup of NT threads.  `sh` needs NT/64 + 1 slots.
// Every thread must call it.  Returns the exclusive prefix; *total gets the
// sum.  Each thread adds up the wave totals itself (a broadcast LDS read),
// so no thread walks them alone between two barriers.
template <typename T, int NT>
__device__ __forceinline__ T block_excl_sum(T v, T* sh, T* total) {
  constexpr int NW = NT / BZG_WAVE;
  const T inc = wave_incl_sum(v);
  const int w = threadIdx.x / BZG_WAVE;
  if (lane() == BZG_WAVE - 1) sh[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) {
    const T t = sh[i];
    before += i < w ? t : T(0);
    all += t;
  }
  *total = all;
  __syncthreads();
  return inc - v + before;
}

// Inclusive max over a workgroup (values must be >= `lo`).
template <typename T, int NT>
__device__ __forceinline__ T block_incl_max(T v, T* sh, T lo) {
  constexpr int NW = NT / BZG_WAVE;
  const T inc = wave_incl_max(v);
  const int w = threadIdx.x / BZG_WAVE;
  if (lane() == BZG_WAVE - 1) sh[w] = inc;
  __syncthreads();
  T before = lo;
#pragma unroll
  for (int i = 0; i < NW; i++) {
    const T t = sh[i];
    before = (i < w && t > before) ? t : before;
  }
  __syncthreads();
  return before > inc ? before : inc;
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
