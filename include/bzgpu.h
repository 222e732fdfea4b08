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
 *    The host copy of the offsets sizes grids and workspace (upper bounds
 *    only); every data-dependent size (RLE1 lengths, block cuts, sort
 *    rounds, symbol counts, stream sizes) stays on the device.
 *  - Every call enqueues its work on `stream` (a hipStream_t; NULL = the
 *    null stream) and returns without waiting for it.  Outputs are valid
 *    once the stream has reached the end of the call's work.
 *  - Return values: 0 when the work was enqueued, a negative BZG_E* code for
 *    an argument or launch error (nothing, or nothing more, is enqueued),
 *    with a message in bzg_last_error().  Errors found by the kernels
 *    themselves (an output range too small, an invalid symbol) are recorded
 *    in the context and reported by bzg_check().  No exception crosses the
 *    ABI.
 *  - d_offsets (device copy of h_offsets, and the other d_* tables) may be
 *    NULL: the library then copies the host table into the workspace
 *    itself (asynchronously, from pinned memory).  Calls that pass every
 *    table and a workspace launch kernels only, and can be captured into a
 *    HIP graph and replayed.
 *  - d_ws/ws_bytes: caller-owned device workspace of at least
 *    bzg_workspace_size() bytes, 256-byte aligned, used until the stream
 *    reaches the end of the call.  d_ws = NULL uses the context's pool, which
 *    grows when needed (stream-ordered: no device-wide synchronisation) and
 *    is shared by every call on the context, in stream order.
 *  - A context may be used by one host thread at a time (calls take a lock
 *    for the time they enqueue).  Calls on different streams may overlap on
 *    the device when each has its own workspace.
 *  - Everything is integer arithmetic; outputs are bit-exact functions of the
 *    inputs (independent of launch sizes, tuning and scheduling).
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
  BZG_EWORKSPACE = -2,/* d_ws smaller than bzg_workspace_size(); size in bzg_last_error() */
  BZG_ECAPACITY = -3, /* (bzg_check) an output range was too small: nothing was packed */
  BZG_EHIP = -4,      /* a HIP runtime call failed; message holds its error string */
  BZG_ENOMEM = -5,    /* device or pinned host allocation failed */
  BZG_EDATA = -6,     /* (bzg_check) inputs inconsistent with each other (a symbol outside the alphabet) */
  BZG_EINTERNAL = -7  /* (bzg_check) a device-side count passed its bound: the results are not valid */
};

/* Call ids for bzg_workspace_size. */
enum { BZG_CALL_BWT = 1, BZG_CALL_MTF = 2, BZG_CALL_HUFFMAN = 3, BZG_CALL_COMPRESS = 4 };

/* Longest block the BWT sort accepts (rows; ranks are kept in 21 bits). */
#define BZG_MAX_BLOCK (1u << 21)

/* Creates a context bound to HIP device `hip_device`.  tune_cache_path
 * (nullable) names a JSON file of tuned launch parameters: its entries for
 * this device and HIP runtime are read now, and bzg_tune adds to it.
 * Returns 0 or BZG_E*. */
int bzg_create(bzg_ctx** out, int hip_device, const char* tune_cache_path);

/* Waits for the device, then releases the context and its pool.  NULL is
 * ignored. */
void bzg_destroy(bzg_ctx* ctx);

/* Message describing the last error on this context ("" if none).  Valid
 * until the next call on the context. */
const char* bzg_last_error(const bzg_ctx* ctx);

/* Waits for `stream`, then reports (and clears) the errors the kernels of
 * calls on this context recorded since the last check: 0, BZG_ECAPACITY,
 * BZG_EDATA or BZG_EINTERNAL (the most serious first), or BZG_EHIP when
 * the stream itself failed. */
int bzg_check(bzg_ctx* ctx, void* stream);

/* Workspace bytes a call needs: call is a BZG_CALL_* id; h_offsets /
 * n_blocks as the call gets them (for BZG_CALL_HUFFMAN the symbol capacity
 * offsets h_sym_offsets); level for BZG_CALL_COMPRESS; n_req the number of
 * streams (1 for compress_blocks).  *bytes receives the size. */
int bzg_workspace_size(bzg_ctx* ctx, int call, const uint64_t* h_offsets, uint32_t n_blocks, int level,
                       uint32_t n_req, size_t* bytes);

/* Upper bound on the stream size compress_blocks can produce for n_bytes of
 * input cut into n_blocks blocks (rounded up to a multiple of 4). */
uint64_t bzg_compress_bound(uint64_t n_bytes, uint32_t n_blocks);

/*
 * Burrows-Wheeler transform of every block (Sec. 3.1): the rotations of the
 * block are sorted as unsigned byte strings, equal rotations by descending
 * start index; d_bwt[off+k] is the byte before rotation k of the sorted
 * order and d_primary[b] the row of rotation 0.  No RLE1 is applied.
 *   d_in       uint8 input; d_in + h_offsets[0] must be 4-byte aligned (text
 *              is read a dword at a time, never past the dword holding the
 *              last byte).
 *   d_offsets  device copy of h_offsets (nullable, see above).
 *   h_offsets  n_blocks+1 host offsets; every block 1..BZG_MAX_BLOCK bytes;
 *              total below 2^32.
 *   d_bwt      uint8 output, same offsets as the input.
 *   d_primary  uint32[n_blocks] output.
 *   d_sa       optional uint32 output (NULL to skip): the sorted rotation start
 *              indices, block-local, same offsets.
 */
int bwt_forward_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                      uint32_t n_blocks, uint8_t* d_bwt, uint32_t* d_primary, uint32_t* d_sa, void* d_ws,
                      size_t ws_bytes, void* stream);

/*
 * Move-to-front (Sec. 3.3) over each block's in-use bytes (the stack starts in
 * ascending byte order) followed by RUNA/RUNB coding of zero runs (bijective
 * base 2, least significant digit first; RUNA=0, RUNB=1), nonzero index v as
 * v+1, and an end-of-block symbol n_inuse+1.
 *   d_bwt      uint8 input blocks at h_offsets (1..BZG_MAX_BLOCK bytes each).
 *   d_syms     uint16 output; block k's symbols start at h_offsets[k] + k and
 *              take at most (block length + 1) slots.
 *   d_nsyms    uint32[n_blocks] output: symbol count per block (EOB included).
 *   d_inuse    uint8[32 * n_blocks] output (4-byte aligned): byte v of block k
 *              is in use iff bit (v & 7) of d_inuse[32k + (v >> 3)] is set.
 */
int mtf_encode_batch(bzg_ctx* ctx, const uint8_t* d_bwt, const uint64_t* d_offsets, const uint64_t* h_offsets,
                     uint32_t n_blocks, uint16_t* d_syms, uint32_t* d_nsyms, uint8_t* d_inuse, void* d_ws,
                     size_t ws_bytes, void* stream);

/*
 * Huffman tables and bit-packing of each block's symbols (Sec. 3.4): 2..6
 * tables chosen per 50-symbol group over four refinement passes, code lengths
 * at most 17, canonical codes; writes the block body in bzip2 syntax (symbol
 * map, table count, selector count, MTF'd unary selectors, delta-coded
 * lengths, codes), MSB first.
 *   d_syms, d_nsyms, d_inuse  as produced by mtf_encode_batch.  A symbol at or
 *                  above the block's alphabet size (in-use bytes + 2), or a
 *                  count above the block's capacity, is reported as BZG_EDATA
 *                  by bzg_check (the body is then not meaningful).
 *   d_sym_offsets / h_sym_offsets  n_blocks+1 offsets: block k's symbols start
 *                  at h_sym_offsets[k]; h_sym_offsets[k+1] bounds its capacity.
 *   d_out          output bytes; block k's body starts at byte h_out_offsets[k]
 *                  and must end before h_out_offsets[k+1].  d_out must be 4-byte
 *                  aligned and the offsets multiples of 4.  Bytes past a body's
 *                  last bit are zero.  A body that does not fit is reported as
 *                  BZG_ECAPACITY by bzg_check and nothing is written.
 *   d_out_offsets  device copy of h_out_offsets (nullable).
 *   d_nbits        uint64[n_blocks] output: body length in bits.
 *   d_tables       optional (NULL to skip) uint8[1568 * n_blocks] output: per
 *                  block, byte 0 = table count G, bytes 16 + 258*t + v = code
 *                  length of symbol v in table t.
 */
int huffman_encode_batch(bzg_ctx* ctx, const uint16_t* d_syms, const uint32_t* d_nsyms, const uint8_t* d_inuse,
                         const uint64_t* d_sym_offsets, const uint64_t* h_sym_offsets, uint32_t n_blocks,
                         uint8_t* d_out, const uint64_t* d_out_offsets, const uint64_t* h_out_offsets,
                         uint64_t* d_nbits, uint8_t* d_tables, void* d_ws, size_t ws_bytes, void* stream);

/*
 * The whole compressor (Sec. 4): block CRC, RLE1, BWT, MTF + RUNA/RUNB,
 * Huffman, packing, and stream assembly into one bzip2 stream with header
 * digit `level` (1..9).  A block whose RLE1 output would exceed 100000*level
 * bytes is cut after the longest prefix whose RLE1 output fits, the rest
 * becoming the next block (and cut again if needed), so every stream
 * respects the decoder limit of its header digit.  Empty blocks are
 * skipped; no bytes gives the 14-byte empty stream.
 *   d_in        uint8 input; blocks at h_offsets (any length; total < 2^31);
 *               may be NULL when every block is empty.
 *   d_out       output stream; out_cap bytes, 4-byte aligned.
 *   d_out_bytes device uint64 output: stream length in bytes.  When the
 *               stream (rounded up to 4 bytes) exceeds out_cap, nothing is
 *               packed, bzg_check reports BZG_ECAPACITY and *d_out_bytes
 *               still holds the length.
 *   d_n_blocks  optional device uint32 output: blocks in the stream.
 */
int compress_blocks(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                    uint32_t n_blocks, int level, uint8_t* d_out, uint64_t out_cap, uint64_t* d_out_bytes,
                    uint32_t* d_n_blocks, void* d_ws, size_t ws_bytes, void* stream);

/*
 * Many independent streams in one pass (Sec. 4: the stages are data-parallel
 * over blocks, so the blocks of several requests are processed together):
 * request r is input blocks [h_req_blocks[r], h_req_blocks[r+1]) and becomes
 * one bzip2 stream of its own, identical to what compress_blocks gives for
 * those blocks alone.  One level for all requests.
 *   d_in, d_offsets, h_offsets, n_blocks  as for compress_blocks (all
 *                  requests' blocks, in request order).
 *   d_req_blocks / h_req_blocks  n_req+1 block indices; [0] = 0,
 *                  [n_req] = n_blocks, non-decreasing.  A request with no
 *                  bytes gets the 14-byte empty stream.  n_req <= 65535.
 *   d_out          output, 4-byte aligned; stream r is written from byte
 *                  h_out_offsets[r] and must end by h_out_offsets[r+1].
 *   d_out_offsets / h_out_offsets  n_req+1 byte offsets, multiples of 4,
 *                  non-decreasing.  Bytes of a range past its stream's
 *                  rounded-up last word are left untouched.
 *   d_out_bytes    device uint64[n_req] output: each stream's length in bytes.
 * When any stream does not fit its range, nothing is packed and bzg_check
 * reports BZG_ECAPACITY (d_out_bytes still filled).
 */
int compress_batch(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                   uint32_t n_blocks, const uint32_t* d_req_blocks, const uint32_t* h_req_blocks, uint32_t n_req,
                   int level, uint8_t* d_out, const uint64_t* d_out_offsets, const uint64_t* h_out_offsets,
                   uint64_t* d_out_bytes, void* d_ws, size_t ws_bytes, void* stream);

/*
 * compress_blocks for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same stream as compress_blocks, with its workspace in a static device
 * array of 128 MiB that the library holds per GPU until the process ends
 * (enough for about 1.5 MB of input; a call that needs more returns
 * BZG_EWORKSPACE with the size in bzg_last_error()).  The call allocates
 * nothing: d_offsets (device copy of h_offsets) is required, and no
 * profiling scopes are recorded.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other contexts,
 * other host threads) race, so a caller serialises them.  The kernels
 * initialise every part of the array they read.  Arguments and results as
 * for compress_blocks.
 */
int compress_blocks_noalloc(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* h_offsets,
                            uint32_t n_blocks, int level, uint8_t* d_out, uint64_t out_cap, uint64_t* d_out_bytes,
                            uint32_t* d_n_blocks, void* stream);

/*
 * Launch parameters.  Three choices change only how the work is spread over
 * the GPU, never a byte of any output: the move-to-front chunk length
 * (mtf_chunk: 2048 or 4096 rows), the Huffman selector groups per
 * assignment tile (assign_groups: 128 or 512) and how many counting steps
 * the small-segment sort may spend per radix pass it saves (count_steps,
 * 1..1024).  0 leaves the built-in choice (which depends on the call's
 * size).  bzg_set_tune fixes them for every later call on the context (all
 * zero: back to the tuned or built-in choices).
 */
int bzg_set_tune(bzg_ctx* ctx, uint32_t mtf_chunk, uint32_t assign_groups, uint32_t count_steps);

/*
 * Autotuning: runs compress_blocks on the given batch at every combination
 * of the launch parameters above (12 points), three times each, checks that
 * every point gives the same stream bytes as the first (BZG_EINTERNAL
 * otherwise), and keeps the fastest for calls of this batch's size bucket
 * (floor(log2 bytes), floor(log2 blocks)) on this context; with a tune cache
 * file (bzg_create) the entry is written there, keyed by the GPU's
 * architecture, the HIP runtime version and the bucket, so later contexts
 * start tuned.  Synchronous; allocates its own output buffers.  h_chosen
 * (nullable) receives {mtf_chunk, assign_groups, count_steps}.
 */
int bzg_tune(bzg_ctx* ctx, const uint8_t* d_in, const uint64_t* h_offsets, uint32_t n_blocks, int level, void* stream,
             uint32_t* h_chosen);

/*
 * Precomputed Huffman tables (Sec. 4: the tables may be computed beforehand
 * by analysing data instead of built per block).  With n_tables = 2..6,
 * every later compress_blocks / compress_batch / compress_host /
 * compress_blocks_noalloc / huffman_encode_batch call on this context codes
 * its blocks with these tables instead of building its own: block b (with
 * alphabet size a = in-use bytes + 2) uses symbols 0..a-2 of each table as
 * given and the length of symbol 257 for its end-of-block symbol; each
 * 50-symbol group takes the table that codes it in the fewest bits (lowest
 * index on ties).  The four refinement passes and every tree build are
 * skipped; the stream stays a standard bzip2 stream (the tables are written
 * into every block as usual).  n_tables = 0 returns to built tables.
 *   h_lens  n_tables rows of 258 code lengths (row stride 258), each 1..17,
 *           each row a prefix code (sum of 2^-len at most 1), so that every
 *           restriction is one too; otherwise BZG_EINVAL.
 * Synchronous: waits for the device, so work already enqueued keeps the
 * tables it was enqueued with.  A table set for a kind of data comes from a
 * sample of it (the Python layer's fixed_tables_from_sample runs the
 * sample's symbols through this library's own table heuristic).
 */
int bzg_set_fixed_tables(bzg_ctx* ctx, const uint8_t* h_lens, int n_tables);

/*
 * Input in host memory, overlapped with the device work (Sec. 2 and Sec. 4:
 * the host link, not the kernels, limits a GPU compressor fed from the
 * host).  The input is cut into blocks of block_bytes (0: 100000*level) and
 * the blocks into chunks of chunk_bytes (rounded down to whole blocks, at
 * least one; 0: 128 blocks).  Each chunk becomes one bzip2 stream, identical
 * to compress_blocks on that chunk's blocks, and the output is the streams
 * one after another (a multi-stream file, which bzip2 decoders read as one).
 * Two device buffers alternate: the upload of chunk i+1 and the download of
 * chunk i-1 run on streams of their own while chunk i is compressed on
 * `stream`.  A pageable h_in is staged through pinned buffers by the host
 * thread; a pinned one (hipHostMalloc) is copied directly.
 *   h_in         n_bytes of input (may be NULL when n_bytes is 0: one empty
 *                stream).
 *   h_out        out_cap bytes of output (pinned or pageable).
 *   h_out_bytes  receives the output length.
 * Unlike the calls above this one is synchronous: it returns once h_out is
 * filled (or with an error: BZG_ECAPACITY when the streams do not fit in
 * out_cap, the device-side errors as bzg_check reports them).  Device
 * buffers of two chunks and their outputs stay with the context for later
 * calls; the workspace comes from the context's pool.
 */
int compress_host(bzg_ctx* ctx, const uint8_t* h_in, uint64_t n_bytes, uint32_t block_bytes, int level,
                  uint64_t chunk_bytes, uint8_t* h_out, uint64_t out_cap, uint64_t* h_out_bytes, void* stream);

/*
 * Decompression on the GPU: one bzip2 stream, or several one after another,
 * back to the original bytes.  Every stage runs on the device: the block
 * and end-of-stream markers are found by a bit-parallel search; each block's
 * Huffman codes, RUNA/RUNB runs and move-to-front list are decoded by one
 * wave (code boundaries are only known serially, Sec. 3.4; the list step is
 * a constant-time lookup, Sec. 3.3); the inverse BWT starts walks of the
 * last-to-first map from many sampled rows and places their pieces by the
 * chain of samples (Sec. 3.1); RLE1 is undone in the Figure 2 pattern (per
 * segment lengths under each incoming state, a scan, then the expansion,
 * Sec. 3.2); every block CRC and stream CRC is checked.
 *   d_in, n_bytes  the compressed bytes (device memory).  Bytes after the
 *                  last stream that do not start another stream are ignored.
 *   d_out          out_cap bytes for the decoded data.
 *   d_out_bytes    device uint64 output: the decoded length.  When it
 *                  exceeds out_cap, nothing is written and bzg_check reports
 *                  BZG_ECAPACITY (*d_out_bytes still holds the length).
 * Unlike the compression calls, this one waits once for the device: the
 * host reads the marker list back to lay the blocks out (and returns
 * BZG_EDATA at once when the input is not a bzip2 stream); the decoding
 * itself is enqueued on `stream` and the call returns without waiting for
 * it.  A stream that does not decode (a bad code, a block that does not end
 * at the next marker, a CRC mismatch, a randomised block) is reported as
 * BZG_EDATA by bzg_check.  The workspace comes from the context's pool.
 */
int decompress(bzg_ctx* ctx, const uint8_t* d_in, uint64_t n_bytes, uint8_t* d_out, uint64_t out_cap,
               uint64_t* d_out_bytes, void* stream);

/*
 * Light-weight field codecs (Sec. 2.1: per-field codes such as null
 * suppression and Elias delta instead of a general-purpose compressor;
 * Sec. 3.5: a GPU float compressor that subtracts a prediction and drops
 * leading zero bytes), built on the same prefix sums as the bzip2 path:
 * every value's code length, a scan to offsets, every code written at its
 * offset (Figure 3).
 *   BZG_FIELD_NS32     uint32 values: 2-bit byte count per value, then the
 *                      significant bytes.
 *   BZG_FIELD_EDELTA32 uint32 values v, coded as the Elias delta code of
 *                      v + 1, with a bit-offset index every 1024 values so
 *                      that decoding runs piece by piece in parallel.
 *   BZG_FIELD_GFC64    doubles (any 64-bit patterns): residual against the
 *                      previous value, sign and leading-zero-byte count in a
 *                      4-bit code, then the remaining bytes; decoding adds
 *                      the residuals up with a scan.
 * The stream layouts are given in fields.hip.  Both calls enqueue on
 * `stream` and take their scratch from the context's pool.
 */
enum { BZG_FIELD_NS32 = 1, BZG_FIELD_EDELTA32 = 2, BZG_FIELD_GFC64 = 3 };

/* Largest stream field_encode can write for n_values values of `codec` (0
 * for an unknown codec). */
uint64_t bzg_field_bound(int codec, uint64_t n_values);

/* d_values: n_values values (uint32, or 8-byte doubles for GFC64), 4- or
 * 8-byte aligned.  d_out: out_cap bytes, 8-byte aligned, at least
 * bzg_field_bound() (else BZG_ECAPACITY before anything is enqueued).
 * d_out_bytes: device uint64 output, the stream length. */
int field_encode(bzg_ctx* ctx, int codec, const void* d_values, uint64_t n_values, uint8_t* d_out, uint64_t out_cap,
                 uint64_t* d_out_bytes, void* stream);

/* d_in: a stream of in_bytes bytes (8-byte aligned) holding n_values values
 * of `codec`; d_values receives them.  A stream whose count or lengths do
 * not fit in_bytes is reported as BZG_EDATA by bzg_check (the output is then
 * not meaningful). */
int field_decode(bzg_ctx* ctx, int codec, const uint8_t* d_in, uint64_t in_bytes, void* d_values, uint64_t n_values,
                 void* stream);

/*
 * Diagnostics: per-kernel timing.  While enabled, every instrumented launch
 * is bracketed by HIP events on its stream, and the device counts that give
 * its algorithmic bytes (the array traffic the method needs, not what the
 * hardware moved) are copied aside; bzg_profile_read waits for the device
 * and adds the launches up per kernel.  bzg_profile(ctx, 1) clears the
 * totals and enables, bzg_profile(ctx, 0) disables.  bzg_profile_read writes
 * one line per kernel, "name launches total_ms total_bytes", NUL-terminated,
 * into buf (cap bytes); BZG_ECAPACITY if it does not fit.
 */
int bzg_profile(bzg_ctx* ctx, int enable);
int bzg_profile_read(bzg_ctx* ctx, char* buf, size_t cap);

#ifdef __cplusplus
}
#endif

#endif /* BZGPU_H */
