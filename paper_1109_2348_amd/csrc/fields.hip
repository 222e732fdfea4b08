// Light-weight field codecs on the prefix-sum primitive: null suppression
// and Elias delta coding of integers (the per-field codes of Sec. 2.1) and a
// GFC-style delta coding of doubles (Sec. 3.5: subtract a prediction, drop
// the leading zero bytes).  Each encoder computes every value's code length,
// turns the lengths into offsets with a scan (per tile, then over the
// tiles), and writes every code at its offset (the Figure 3 pattern); the
// decoders invert it the same way (Elias delta, whose lengths are only known
// by decoding, keeps an index of every 1024th value's bit offset and decodes
// the 1024-value pieces in parallel).
//
// Stream layouts (the value count n first, as a little-endian uint64):
//   NS32    n; 2-bit codes (bytes - 1), four per byte, low bits first; the
//           values' significant bytes, least significant first.
//   EDELTA  n; total bits; bit offset of every 1024th value (uint64 each);
//           the codes of v + 1 back to back, bit k of the stream being bit
//           31 - k % 32 of 32-bit word k / 32.
//   GFC64   n; 4-bit codes (sign << 3 | leading zero bytes, at most 7), two
//           per byte, low nibble first; each residual's 8 - lzb low bytes.
#include "../../include/bzgpu.h"
#include "common.hpp"
#include "internal.hpp"
#include "plan.hpp"

namespace bzg {

constexpr uint32_t FPER = 16;              // values per thread
constexpr uint32_t FTILE = NT * FPER;      // values per workgroup tile
constexpr uint32_t EDELTA_EVERY = 1024;    // index granularity of Elias delta

// ------------------------------------------------------------- lengths

__device__ __forceinline__ uint32_t ns_len(uint32_t v) {
  return v < (1u << 8) ? 1u : v < (1u << 16) ? 2u : v < (1u << 24) ? 3u : 4u;
}
// Elias delta of x = v + 1: N = floor(log2 x), M = floor(log2(N + 1)).
__device__ __forceinline__ uint32_t ed_len(uint32_t v) {
  const uint64_t x = (uint64_t)v + 1;
  const uint32_t N = 63u - (uint32_t)__clzll((long long)x);
  const uint32_t M = 31u - (uint32_t)__clz(N + 1);
  return N + 2 * M + 1;
}
// GFC residual: magnitude, sign flag and leading zero bytes (at most 7).
__device__ __forceinline__ void gfc_res(uint64_t w, uint64_t prev, uint64_t& mag, uint32_t& code) {
  uint64_t r = w - prev;
  const uint32_t sign = (uint32_t)(r >> 63);
  if (sign) r = 0ull - r;
  const uint32_t lz = r ? (uint32_t)__clzll((long long)r) : 64u;
  const uint32_t lzb = min(lz / 8, 7u);
  mag = r;
  code = (sign << 3) | lzb;
}

// Length of value i under codec c (from the values for the encoders, from
// the code region for the NS32 / GFC64 decoders).
__device__ __forceinline__ uint32_t enc_len(int c, const void* vals, uint64_t i) {
  if (c == BZG_FIELD_NS32) return ns_len(((const uint32_t*)vals)[i]);
  if (c == BZG_FIELD_EDELTA32) return ed_len(((const uint32_t*)vals)[i]);
  const uint64_t* w = (const uint64_t*)vals;
  uint64_t mag;
  uint32_t code;
  gfc_res(w[i], i ? w[i - 1] : 0ull, mag, code);
  return 8u - (code & 7u);
}
__device__ __forceinline__ uint32_t dec_len(int c, const uint8_t* codes, uint64_t i) {
  if (c == BZG_FIELD_NS32) return ((codes[i >> 2] >> (2 * (i & 3))) & 3u) + 1u;
  return 8u - ((codes[i >> 1] >> (4 * (i & 1))) & 7u);
}

// ------------------------------------------------------------ scans

// Pass over tiles: the sum of the lengths (or, decode == 2, of the GFC
// residuals) of every tile.
__global__ __launch_bounds__(NT) void k_field_sums(int c, int decode, const void* __restrict__ src, uint64_t n,
                                                   uint64_t in_bytes, const uint64_t* __restrict__ byte_off,
                                                   uint64_t* __restrict__ tile_sum) {
  __shared__ uint64_t sh[NT / BZG_WAVE + 1];
  const uint64_t i0 = ((uint64_t)blockIdx.x * NT + threadIdx.x) * FPER;
  uint64_t s = 0;
  // GFC residuals, from their byte offsets (when the bytes are all there)
  if (decode == 2 && byte_off[gridDim.x] <= in_bytes - 8 - (n + 1) / 2) {
    const uint8_t* z = (const uint8_t*)src;
    const uint8_t* codes = z + 8;
    const uint8_t* data = codes + (n + 1) / 2;
    uint64_t off = byte_off[blockIdx.x];
    uint32_t lens[FPER];
    uint32_t tl = 0;
#pragma unroll
    for (uint32_t k = 0; k < FPER; k++) {
      lens[k] = i0 + k < n ? dec_len(c, codes, i0 + k) : 0u;
      tl += lens[k];
    }
    uint64_t tot;
    off += block_excl_sum<uint64_t, NT>(tl, sh, &tot);
    for (uint32_t k = 0; k < FPER; k++) {
      if (i0 + k >= n) break;
      uint64_t r = 0;
      for (uint32_t b = 0; b < lens[k]; b++) r |= (uint64_t)data[off + b] << (8 * b);
      const uint32_t code = (codes[(i0 + k) >> 1] >> (4 * ((i0 + k) & 1))) & 15u;
      s += (code >> 3) ? 0ull - r : r;
      off += lens[k];
    }
  } else if (decode < 2) {
    for (uint32_t k = 0; k < FPER; k++) {
      const uint64_t i = i0 + k;
      if (i < n) s += decode ? dec_len(c, (const uint8_t*)src + 8, i) : enc_len(c, src, i);
    }
  }
  const uint64_t t = block_sum<uint64_t, NT>(s, sh);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = t;
}

// Exclusive scan of m tile sums in one workgroup of 1024 threads (modulo
// 2^64); out[m] = the total.
__global__ __launch_bounds__(1024) void k_field_tscan(const uint64_t* __restrict__ in, uint32_t m,
                                                      uint64_t* __restrict__ out) {
  __shared__ uint64_t sh[1024 / BZG_WAVE + 1];
  const uint32_t per = (m + 1023) / 1024, lo = min(threadIdx.x * per, m), hi = min(lo + per, m);
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; i++) s += in[i];
  uint64_t tot;
  uint64_t run = block_excl_sum<uint64_t, 1024>(s, sh, &tot);
  for (uint32_t i = lo; i < hi; i++) {
    out[i] = run;
    run += in[i];
  }
  if (threadIdx.x == 0) out[m] = tot;
}

// ---------------------------------------------------------- encoders

// Writes every value's code: codes (NS32 / GFC64) and bytes at their
// offsets, or (EDELTA) the bit codes OR-ed into the zeroed stream words and
// the index entries.  The header is written by the first thread.
__global__ __launch_bounds__(NT) void k_field_encode(int c, const void* __restrict__ vals, uint64_t n,
                                                     const uint64_t* __restrict__ tile_off, uint8_t* __restrict__ out,
                                                     uint64_t* __restrict__ out_bytes) {
  __shared__ uint64_t sh[NT / BZG_WAVE + 1];
  const uint64_t tid = (uint64_t)blockIdx.x * NT + threadIdx.x, i0 = tid * FPER;
  uint32_t lens[FPER];
  uint32_t tl = 0;
#pragma unroll
  for (uint32_t k = 0; k < FPER; k++) {
    lens[k] = i0 + k < n ? enc_len(c, vals, i0 + k) : 0u;
    tl += lens[k];
  }
  uint64_t tot;
  uint64_t off = tile_off[blockIdx.x] + block_excl_sum<uint64_t, NT>(tl, sh, &tot);
  const uint32_t nt = gridDim.x;
  if (tid == 0) {
    ((uint64_t*)out)[0] = n;
    if (c == BZG_FIELD_EDELTA32) ((uint64_t*)out)[1] = tile_off[nt];
  }
  if (c == BZG_FIELD_EDELTA32) {
    const uint64_t ni = (n + EDELTA_EVERY - 1) / EDELTA_EVERY;
    uint64_t* index = (uint64_t*)out + 2;
    uint32_t* words = (uint32_t*)(index + ni);
    if (tid == 0) *out_bytes = 16 + 8 * ni + 4 * ((tile_off[nt] + 31) / 32);
    const uint32_t* v = (const uint32_t*)vals;
    for (uint32_t k = 0; k < FPER; k++) {
      const uint64_t i = i0 + k;
      if (i >= n) break;
      if (i % EDELTA_EVERY == 0) index[i / EDELTA_EVERY] = off;
      const uint64_t x = (uint64_t)v[i] + 1;
      const uint32_t N = 63u - (uint32_t)__clzll((long long)x), len = lens[k];
      const uint64_t code = ((uint64_t)(N + 1) << N) | (x - (1ull << N));  // M leading zeros are implicit
      const uint64_t a = code << (64 - len);  // left-aligned
      const uint64_t w = off >> 5;
      const uint32_t s = (uint32_t)(off & 31);
      const uint64_t hi = a >> s;
      const uint32_t w0 = (uint32_t)(hi >> 32), w1 = (uint32_t)hi, w2 = s ? (uint32_t)((a << (64 - s)) >> 32) : 0u;
      if (w0) atomicOr(&words[w], w0);
      if (w1) atomicOr(&words[w + 1], w1);
      if (w2) atomicOr(&words[w + 2], w2);
      off += len;
    }
    return;
  }
  const uint64_t ncode = c == BZG_FIELD_NS32 ? (n + 3) / 4 : (n + 1) / 2;
  uint8_t* codes = out + 8;
  uint8_t* data = codes + ncode;
  if (tid == 0) *out_bytes = 8 + ncode + tile_off[nt];
  if (c == BZG_FIELD_NS32) {
    const uint32_t* v = (const uint32_t*)vals;
    uint32_t cw = 0;
    for (uint32_t k = 0; k < FPER; k++) {
      const uint64_t i = i0 + k;
      if (i >= n) break;
      cw |= (lens[k] - 1) << (2 * k);
      for (uint32_t b = 0; b < lens[k]; b++) data[off + b] = (uint8_t)(v[i] >> (8 * b));
      off += lens[k];
    }
    // four code bytes per thread (byte-wise where the code region ends)
    for (uint32_t b = 0; b < 4; b++)
      if (i0 / 4 + b < ncode) codes[i0 / 4 + b] = (uint8_t)(cw >> (8 * b));
  } else {
    const uint64_t* w = (const uint64_t*)vals;
    uint64_t cw = 0;
    for (uint32_t k = 0; k < FPER; k++) {
      const uint64_t i = i0 + k;
      if (i >= n) break;
      uint64_t mag;
      uint32_t code;
      gfc_res(w[i], i ? w[i - 1] : 0ull, mag, code);
      cw |= (uint64_t)code << (4 * k);
      for (uint32_t b = 0; b < lens[k]; b++) data[off + b] = (uint8_t)(mag >> (8 * b));
      off += lens[k];
    }
    for (uint32_t b = 0; b < 8; b++)
      if (i0 / 2 + b < ncode) codes[i0 / 2 + b] = (uint8_t)(cw >> (8 * b));
  }
}

// ---------------------------------------------------------- decoders

// NS32 / GFC64: every value from its bytes; GFC adds the residuals up (its
// tile carries come from the scan of the tiles' residual sums).
__global__ __launch_bounds__(NT) void k_field_decode(int c, const uint8_t* __restrict__ z, uint64_t in_bytes,
                                                     uint64_t n, const uint64_t* __restrict__ byte_off,
                                                     const uint64_t* __restrict__ res_off, void* __restrict__ vals,
                                                     uint32_t* __restrict__ err) {
  __shared__ uint64_t sh[NT / BZG_WAVE + 1];
  const uint64_t tid = (uint64_t)blockIdx.x * NT + threadIdx.x, i0 = tid * FPER;
  const uint64_t ncode = c == BZG_FIELD_NS32 ? (n + 3) / 4 : (n + 1) / 2;
  const uint8_t* codes = z + 8;
  const uint8_t* data = codes + ncode;
  const uint64_t avail = in_bytes - 8 - ncode;  // the caller checked in_bytes > 8 + ncode
  uint32_t lens[FPER];
  uint32_t tl = 0;
#pragma unroll
  for (uint32_t k = 0; k < FPER; k++) {
    lens[k] = i0 + k < n ? dec_len(c, codes, i0 + k) : 0u;
    tl += lens[k];
  }
  uint64_t tot;
  uint64_t off = byte_off[blockIdx.x] + block_excl_sum<uint64_t, NT>(tl, sh, &tot);
  if (tid == 0 && (byte_off[gridDim.x] > avail || ((const uint64_t*)z)[0] != n)) atomicOr(err, ERR_STREAM);
  if (byte_off[gridDim.x] > avail) return;
  if (c == BZG_FIELD_NS32) {
    uint32_t* v = (uint32_t*)vals;
    for (uint32_t k = 0; k < FPER; k++) {
      const uint64_t i = i0 + k;
      if (i >= n) break;
      uint32_t x = 0;
      for (uint32_t b = 0; b < lens[k]; b++) x |= (uint32_t)data[off + b] << (8 * b);
      v[i] = x;
      off += lens[k];
    }
    return;
  }
  // GFC: residuals of this thread, their in-tile prefix, plus the carry
  uint64_t r[FPER];
  uint64_t rs = 0;
#pragma unroll
  for (uint32_t k = 0; k < FPER; k++) {
    uint64_t m = 0;
    for (uint32_t b = 0; b < lens[k]; b++) m |= (uint64_t)data[off + b] << (8 * b);
    off += lens[k];
    const uint32_t code = i0 + k < n ? (codes[(i0 + k) >> 1] >> (4 * ((i0 + k) & 1))) & 15u : 0u;
    r[k] = (code >> 3) ? 0ull - m : m;
    rs += r[k];
  }
  uint64_t t2;
  uint64_t acc = res_off[blockIdx.x] + block_excl_sum<uint64_t, NT>(rs, sh, &t2);
  uint64_t* v = (uint64_t*)vals;
#pragma unroll
  for (uint32_t k = 0; k < FPER; k++) {
    acc += r[k];
    if (i0 + k < n) v[i0 + k] = acc;
  }
}

// Elias delta: one thread per indexed piece of up to 1024 values.
__global__ __launch_bounds__(NT) void k_edelta_decode(const uint8_t* __restrict__ z, uint64_t in_bytes, uint64_t n,
                                                      uint32_t* __restrict__ vals, uint32_t* __restrict__ err) {
  const uint64_t p = (uint64_t)blockIdx.x * NT + threadIdx.x;
  const uint64_t ni = (n + EDELTA_EVERY - 1) / EDELTA_EVERY;
  if (p >= ni) return;
  const uint64_t total = ((const uint64_t*)z)[1];
  const uint64_t* index = (const uint64_t*)z + 2;
  const uint32_t* words = (const uint32_t*)(index + ni);
  const uint64_t nw = (total + 31) / 32;
  if (16 + 8 * ni + 4 * nw > in_bytes) {
    atomicOr(err, ERR_STREAM);
    return;
  }
  auto word = [&](uint64_t k) -> uint64_t { return k < nw ? words[k] : 0u; };
  // the 64 stream bits from bit q on
  auto bits64 = [&](uint64_t q) -> uint64_t {
    const uint64_t k = q >> 5;
    const uint32_t s = (uint32_t)(q & 31);
    const uint64_t hi = (word(k) << 32) | word(k + 1);
    return s ? (hi << s) | (word(k + 2) >> (32 - s)) : hi;
  };
  uint64_t q = index[p];
  const uint64_t lo = p * EDELTA_EVERY, hi = min(lo + EDELTA_EVERY, n);
  for (uint64_t i = lo; i < hi; i++) {
    const uint64_t a = bits64(q);
    const uint32_t M = a ? (uint32_t)__clzll((long long)a) : 64u;
    if (M > 5 || q + 2 * M + 1 > total) {
      atomicOr(err, ERR_STREAM);
      return;
    }
    const uint32_t N = (uint32_t)(a >> (64 - (2 * M + 1))) - 1;  // the M + 1 bits of N + 1
    if (N > 32) {
      atomicOr(err, ERR_STREAM);
      return;
    }
    const uint64_t b = bits64(q + 2 * M + 1);
    const uint64_t low = N ? b >> (64 - N) : 0ull;
    vals[i] = (uint32_t)(((1ull << N) | low) - 1);
    q += N + 2 * M + 1;
  }
}

// ---------------------------------------------------------- launchers

uint64_t field_bound(int c, uint64_t n) {
  if (c == BZG_FIELD_NS32) return 8 + (n + 3) / 4 + 4 * n + 16;
  if (c == BZG_FIELD_EDELTA32) return 16 + 8 * ((n + EDELTA_EVERY - 1) / EDELTA_EVERY) + 4 * ((43 * n + 31) / 32) + 16;
  return 8 + (n + 1) / 2 + 8 * n + 16;
}
uint64_t field_tiles(uint64_t n) { return std::max<uint64_t>((n + FTILE - 1) / FTILE, 1); }

hipError_t field_encode_run(int c, const void* vals, uint64_t n, uint8_t* out, uint64_t* out_bytes,
                            uint64_t* tile_sum, uint64_t* tile_off, hipStream_t st) {
  const uint32_t nt = (uint32_t)field_tiles(n);
  ProfScope ps("field_encode", st, (double)n * (c == BZG_FIELD_GFC64 ? 8 : 4));
  hipLaunchKernelGGL(k_field_sums, dim3(nt), dim3(NT), 0, st, c, 0, vals, n, (uint64_t)0, nullptr, tile_sum);
  hipLaunchKernelGGL(k_field_tscan, dim3(1), dim3(1024), 0, st, tile_sum, nt, tile_off);
  if (c == BZG_FIELD_EDELTA32) {  // the bit stream is OR-ed into zeroed words
    const uint64_t ni = (n + EDELTA_EVERY - 1) / EDELTA_EVERY;
    const uint64_t words = (43 * n + 31) / 32 + 3;
    hipError_t e = fill32((uint32_t*)(out + 16 + 8 * ni), words, 0u, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_field_encode, dim3(nt), dim3(NT), 0, st, c, vals, n, tile_off, out, out_bytes);
  return hipGetLastError();
}

hipError_t field_decode_run(int c, const uint8_t* z, uint64_t in_bytes, uint64_t n, void* vals, uint64_t* tile_sum,
                            uint64_t* byte_off, uint64_t* res_sum, uint64_t* res_off, uint32_t* err,
                            hipStream_t st) {
  ProfScope ps("field_decode", st, (double)n * (c == BZG_FIELD_GFC64 ? 8 : 4));
  if (c == BZG_FIELD_EDELTA32) {
    const uint64_t ni = (n + EDELTA_EVERY - 1) / EDELTA_EVERY;
    hipLaunchKernelGGL(k_edelta_decode, dim3((uint32_t)std::max<uint64_t>((ni + NT - 1) / NT, 1)), dim3(NT), 0, st,
                       z, in_bytes, n, (uint32_t*)vals, err);
    return hipGetLastError();
  }
  const uint32_t nt = (uint32_t)field_tiles(n);
  hipLaunchKernelGGL(k_field_sums, dim3(nt), dim3(NT), 0, st, c, 1, z, n, in_bytes, nullptr, tile_sum);
  hipLaunchKernelGGL(k_field_tscan, dim3(1), dim3(1024), 0, st, tile_sum, nt, byte_off);
  if (c == BZG_FIELD_GFC64) {
    hipLaunchKernelGGL(k_field_sums, dim3(nt), dim3(NT), 0, st, c, 2, z, n, in_bytes, byte_off, res_sum);
    hipLaunchKernelGGL(k_field_tscan, dim3(1), dim3(1024), 0, st, res_sum, nt, res_off);
  }
  hipLaunchKernelGGL(k_field_decode, dim3(nt), dim3(NT), 0, st, c, z, in_bytes, n, byte_off,
                     c == BZG_FIELD_GFC64 ? res_off : byte_off, vals, err);
  return hipGetLastError();
}

}  // namespace bzg
