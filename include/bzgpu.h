/*
 * bzgpu -- batched bzip2 compression stages on one AMD Instinct MI355X
 * (gfx950), behind a plain C ABI.
 *
 * The stages follow "Lossless data compression on GPGPU architectures"
 * (Eirola): the Burrows-Wheeler transform as a sort of the rotations of each
 * block (Sec. 3.1), move-to-front over a stack of recently used symbols
 * (Sec. 3.3), variable-length (Huffman) coding with codes placed at the
 * prefix sum of their lengths (Sec. 3.4, Figure 3), combined into a
 * bzip2-compatible compressor that keeps all data on the device (Sec. 4).
 * Run-length coding (Sec. 3.2, Figure 1) appears as bzip2's RLE1 and its
 * RUNA/RUNB zero-run coding.
 *
 * Conventions shared by every call:
 *  - d_* pointers are device memory owned by the caller; h_* pointers are host
 *    memory owned by the caller and only read during the call.  The library
 *    never frees caller memory.
 *  - A batch of blocks is one concatenated buffer plus offsets: block k is
 *    bytes [h_offsets[k], h_offsets[k+1]).  Offsets must be nondecreasing.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    The calls synchronise `stream` internally where the next launch depends
 *    on a data-dependent size (one small device-to-host copy per sorting round
 *    and per planning step); outputs are complete when the call returns 0.
 *  - Return values: 0 on success, a negative BZG_E* code otherwise, with a
 *    message in bzg_last_error().  No exception crosses the ABI.
 *  - Calls on one context run one at a time (the context holds a lock for
 *    the whole call); to overlap work from several host threads give each
 *    thread its own context and stream.  Scratch memory is owned by the
 *    context and grows on demand (hipMalloc); it is released by
 *    bzg_destroy().  bzg_last_error() gives the message of the latest
 *    call on the context.
 *  - Everything is integer arithmetic; outputs are bit-exact functions of the
 *    inputs (independent of launch sizes and scheduling).
 */
#ifndef BZGPU_H
#define BZGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bzg_ctx bzg_ctx;

enum {
  BZG_OK = 0,
  BZG_EINVAL = -1,    /* bad argument: null pointer, bad offsets, block too long */
  BZG_ECAPACITY = -3, /* an output buffer is too small; see bzg_last_error() */
  BZG_EHIP = -4,      /* a HIP runtime call failed; message holds its error string */
  BZG_ENOMEM = -5,    /* device or pinned host allocation failed */
  BZG_EDATA = -6      /* inputs inconsistent with each other (e.g. a symbol outside the alphabet) */
};

/* Longest block the BWT sort accepts (rows; ranks are kept in 21 bits). */
#define BZG_MAX_BLOCK (1u << 21)

/* Creates a context bound to HIP device `hip_device`.  Returns 0 or BZG_E*. */
int bzg_create(bzg_ctx** out, int hip_device);

/* Releases the context and its scratch memory.  NULL is ignored. */
void bzg_destroy(bzg_ctx* ctx);

/* Message describing the last error on this context ("" if none).  Valid
 * until the next call on the context. */
const char* bzg_last_error(const bzg_ctx* ctx);

/* Upper bound on the stream size compress_blocks can produce for n_bytes of
 * input cut into n_blocks blocks (rounded up to a multiple of 4). */
uint64_t bzg_compress_bound(uint64_t n_bytes, uint32_t n_blocks);

/*
 * Burrows-Wheeler transform of every block (Sec. 3.1): the rotations of the
 * block are sorted as unsigned byte strings, equal rotations by descending
 * start index; d_bwt[off+k] is the byte before rotation k of the sorted
 * order and d_primary[b] the row of rotation 0.  No RLE1 is applied.
 *   d_in       uint8 input, h_offsets[n_blocks] bytes.
 *   h_offsets  n_blocks+1 host offsets; every block 1..BZG_MAX_BLOCK bytes;
 *              total below 2^32.
 *   d_bwt      uint8 output, same offsets as the input.
 *   d_primary  uint32[n_blocks] output.
 *   d_sa       optional uint32 output (NULL to skip): the sorted rotation start
 *              indices, block-local, same offsets.
 */
int bwt_forward_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks,
                      uint8_t* d_bwt, uint32_t* d_primary, uint32_t* d_sa, void* stream);

/*
 * Move-to-front (Sec. 3.3) over each block's in-use bytes (the stack starts in
 * ascending byte order) followed by RUNA/RUNB coding of zero runs (bijective
 * base 2, least significant digit first; RUNA=0, RUNB=1), nonzero index v as
 * v+1, and an end-of-block symbol n_inuse+1.
 *   d_bwt      uint8 input blocks at h_offsets (1..BZG_MAX_BLOCK bytes each).
 *   d_syms     uint16 output; block k's symbols start at h_offsets[k] + k and
 *              take at most (block length + 1) slots.
 *   d_nsyms    uint32[n_blocks] output: symbol count per block (EOB included).
 *   d_inuse    uint8[32 * n_blocks] output: byte v of block k is in use iff
 *              bit (v & 7) of d_inuse[32k + (v >> 3)] is set.
 */
int mtf_encode_batch(bzg_ctx* ctx, const uint8_t* d_bwt, const uint64_t* h_offsets, uint32_t n_blocks,
                     uint16_t* d_syms, uint32_t* d_nsyms, uint8_t* d_inuse, void* stream);

/*
 * Huffman tables and bit-packing of each block's symbols (Sec. 3.4): 2..6
 * tables chosen per 50-symbol group over four refinement passes, code lengths
 * at most 17, canonical codes; writes the block body in bzip2 syntax (symbol
 * map, table count, selector count, MTF'd unary selectors, delta-coded
 * lengths, codes), MSB first.
 *   d_syms, d_nsyms, d_inuse  as produced by mtf_encode_batch.
 *   h_sym_offsets  n_blocks+1 host offsets: block k's symbols start at
 *                  h_sym_offsets[k]; h_sym_offsets[k+1] bounds its capacity.
 *   d_out          output bytes; block k's body starts at byte h_out_offsets[k]
 *                  and must end before h_out_offsets[k+1].  d_out must be 4-byte
 *                  aligned and h_out_offsets[n_blocks] a multiple of 4.  Bytes
 *                  past a body's last bit are zero.
 *   d_nbits        uint64[n_blocks] output: body length in bits.
 *   d_tables       optional (NULL to skip) uint8[1568 * n_blocks] output: per
 *                  block, byte 0 = table count G, bytes 16 + 258*t + v = code
 *                  length of symbol v in table t.
 */
int huffman_encode_batch(bzg_ctx* ctx, const uint16_t* d_syms, const uint32_t* d_nsyms, const uint8_t* d_inuse,
                         const uint64_t* h_sym_offsets, uint32_t n_blocks, uint8_t* d_out,
                         const uint64_t* h_out_offsets, uint64_t* d_nbits, uint8_t* d_tables, void* stream);

/*
 * The whole compressor (Sec. 4): block CRC, RLE1, BWT, MTF + RUNA/RUNB,
 * Huffman, packing, and stream assembly into one bzip2 stream with header
 * digit `level` (1..9).  A block whose RLE1 output would exceed 100000*level
 * bytes is cut after the longest prefix whose RLE1 output fits, the rest
 * becoming the next block, so every stream respects the decoder limit of its
 * header digit.  Empty blocks are skipped; no blocks gives the 14-byte empty
 * stream.
 *   d_in        uint8 input; blocks at h_offsets (any length; total < 2^31);
 *               may be NULL when every block is empty.
 *   d_out       output stream; out_cap bytes, 4-byte aligned.
 *   h_out_bytes host uint64 output: stream length in bytes (also set when
 *               BZG_ECAPACITY is returned; the capacity needed is that
 *               rounded up to a multiple of 4).
 *   h_n_blocks  optional host uint32 output: blocks in the stream.
 */
int compress_blocks(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks, int level,
                    uint8_t* d_out, uint64_t out_cap, uint64_t* h_out_bytes, uint32_t* h_n_blocks, void* stream);

/*
 * Many independent streams in one pass (Sec. 4: the stages are data-parallel
 * over blocks, so the blocks of several requests are processed together):
 * request r is input blocks [h_req_blocks[r], h_req_blocks[r+1]) and becomes
 * one bzip2 stream of its own, identical to what compress_blocks gives for
 * those blocks alone.  One level for all requests.
 *   d_in, h_offsets, n_blocks  as for compress_blocks (all requests' blocks,
 *                  in request order).
 *   h_req_blocks   n_req+1 host block indices; [0] = 0, [n_req] = n_blocks,
 *                  non-decreasing.  A request with no bytes gets the 14-byte
 *                  empty stream.  n_req <= 65535.
 *   d_out          output, 4-byte aligned; stream r is written from byte
 *                  h_out_offsets[r] and must end by h_out_offsets[r+1].
 *   h_out_offsets  n_req+1 host byte offsets, multiples of 4, non-decreasing.
 *                  Bytes of a range past its stream's rounded-up last word
 *                  are left untouched.
 *   h_out_bytes    host uint64[n_req] output: each stream's length in bytes.
 * Returns BZG_ECAPACITY (h_out_bytes still filled; nothing packed) when a
 * stream, rounded up to 4 bytes, does not fit its range.
 */
int compress_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks,
                   const uint32_t* h_req_blocks, uint32_t n_req, int level, uint8_t* d_out,
                   const uint64_t* h_out_offsets, uint64_t* h_out_bytes, void* stream);

/*
 * Diagnostics: per-kernel timing.  While enabled, every instrumented launch
 * is bracketed by HIP events on its stream; after each call the elapsed times
 * are added up per kernel together with the launch's algorithmic bytes (the
 * array traffic the method needs, not what the hardware moved).
 * bzg_profile(ctx, 1) clears the totals and enables, bzg_profile(ctx, 0)
 * disables.  bzg_profile_read writes one line per kernel,
 * "name launches total_ms total_bytes", NUL-terminated, into buf (cap bytes);
 * BZG_ECAPACITY if it does not fit.
 */
int bzg_profile(bzg_ctx* ctx, int enable);
int bzg_profile_read(bzg_ctx* ctx, char* buf, size_t cap);

#ifdef __cplusplus
}
#endif

#endif /* BZGPU_H */
