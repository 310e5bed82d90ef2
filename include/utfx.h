/*
 * utfx.h -- validating UTF-8 <-> UTF-16LE transcoding on AMD Instinct MI355X (gfx950),
 * with UTF-16BE and UTF-32LE forms, batched calls, graphs, a server and streams.
 *
 * The operations are those of Clausecker & Lemire, "Transcoding Unicode Characters
 * with AVX-512 Instructions": validating transcoding that, on the first encoding
 * error, transcodes the characters before it and stops, reporting where (sections
 * 6.4 and 7.4), with the output length reported to the caller (section 7.5).  Each
 * direction also has a validate-only call and an output-length query.
 *
 * Memory: every data pointer passed to these calls (in, out, results, item tables,
 * arenas) is a DEVICE pointer (for example a torch tensor's data_ptr()).  The caller
 * owns all of them; the library never allocates on a call.  The context owns its
 * workspace (a status word per tile, a few counters), a device result slot and a
 * pinned host copy of it.
 *
 * Threading: one context per HIP stream.  Calls on a context run in stream order;
 * synchronous calls block the calling thread until their own result is on the host.
 * Two contexts may run concurrently on different streams.
 *
 * Alignment: UTF-8 input and output may start at any byte address.  UTF-16 pointers
 * must be 2-byte aligned and UTF-32 pointers 4-byte aligned (else UTFX_E_INVALID_ARG).
 * Lengths are in code units: bytes for UTF-8, 16-bit words for UTF-16, 32-bit units for
 * UTF-32.
 *
 * Result (every call): see utfx_result.  Precedence: argument error, then the
 * earliest encoding error, then UTFX_E_OUTPUT_TOO_SMALL, then UTFX_OK.  n = 0 is OK
 * with count 0.
 */
#ifndef UTFX_H
#define UTFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct utfx_ctx utfx_ctx;

typedef enum {
  UTFX_OK = 0,
  /* UTF-8 error kinds.  The paper reports a position only; the kind is the first
   * validation rule of section 6.4 that the character starting at the offset breaks,
   * checked as: byte type, continuation bytes present, shortest form, surrogate,
   * U+10FFFF bound. */
  UTFX_E_STRAY_CONT = 1,   /* continuation byte where a character must start (rule 3) */
  UTFX_E_MISSING_CONT = 2, /* lead byte not followed by its continuation bytes, including
                              by the end of the input (rule 2) */
  UTFX_E_OVERLONG = 3,     /* C0/C1, or a 3- or 4-byte form below its minimum (rule 4) */
  UTFX_E_TOO_LARGE = 4,    /* F4 form above U+10FFFF (rule 5) */
  UTFX_E_SURROGATE = 5,    /* UTF-8: encoded U+D800..DFFF (rule 6); UTF-16: a high surrogate
                              not followed by a low one, or a low one not preceded by a high
                              one (sections 2.1 and 7.4) */
  UTFX_E_BAD_BYTE = 6,     /* byte F5..FF (rule 1) */
  UTFX_E_OUTPUT_TOO_SMALL = 16, /* input valid, but the output needs more than cap units */
  UTFX_E_INVALID_ARG = 17,      /* null pointer with n > 0, misaligned UTF-16 pointer,
                                   n above UTFX_MAX_UNITS, bad batch descriptor */
  UTFX_E_DEVICE = 18            /* HIP runtime failure or a watchdog trip; see
                                   utfx_last_error() */
} utfx_status;

/* 24-byte call result.
 *   status   utfx_status
 *   count    OK: units written (transcode), n (validate), output length (length query);
 *            encoding error: offset, in input units, of the first invalid unit;
 *            OUTPUT_TOO_SMALL: output units the input needs
 *   written  transcode: output units of the valid prefix in[0:count]; those are in
 *            out[0:min(written, cap)].  On OUTPUT_TOO_SMALL it is 0.
 *            validate and length query: equal to count.
 * Output beyond `written` is unspecified (but nothing is stored at or beyond cap). */
typedef struct {
  int32_t status;
  uint32_t reserved;
  uint64_t count;
  uint64_t written;
} utfx_result;

/* Largest n accepted by any call (input units). */
#define UTFX_MAX_UNITS (((uint64_t)1) << 35)

/* ---- context ------------------------------------------------------------------- */

/* Creates a context bound to `hip_stream` (a hipStream_t; NULL = the default stream)
 * on the current device.  Allocates the workspace once.  Returns UTFX_OK or
 * UTFX_E_DEVICE.  *ctx is NULL on failure. */
utfx_status utfx_create(utfx_ctx **ctx, void *hip_stream);
/* Destroys the context after draining its stream.  NULL is a no-op. */
void utfx_destroy(utfx_ctx *ctx);
/* Text of the last error on this context ("" if none).  Valid until the next call. */
const char *utfx_last_error(const utfx_ctx *ctx);
/* Rebinds the context to another stream (work already queued stays where it is). */
utfx_status utfx_set_stream(utfx_ctx *ctx, void *hip_stream);
/* Kernel timing.  While set, every single-buffer call on the context records
 * start_event (a hipEvent_t) on its stream immediately before its main kernel and
 * stop_event immediately after it (hipExtLaunchKernel), so that hipEventElapsedTime
 * gives that kernel's own duration, without the finalisation kernel and the gaps
 * between launches.  NULL, NULL switches it off; nothing is recorded while capturing
 * a graph.  UTFX_E_INVALID_ARG if only one of the two is NULL.  The events stay owned
 * by the caller and must outlive their use. */
utfx_status utfx_set_kernel_events(utfx_ctx *ctx, void *start_event, void *stop_event);

/* Tunables of one operation, picked by the autotuner.  op is a utfx_op.
 * tile_bytes: input bytes one workgroup handles per step (4096 or 8192: 16 bytes per
 *             thread, so 256 or 512 threads);
 * tiles_per_segment: tiles per workgroup (1..256); a workgroup owns one segment of
 *             tile_bytes * tiles_per_segment input bytes and performs one cross-
 *             segment look-back for it.  The transcodes hold a whole segment in
 *             registers and its output in LDS, so they take only these pairs:
 *             UTF-8 -> UTF-16 (4096, 2, 4 or 8), (8192, 2 or 4); UTF-16 -> UTF-8
 *             (4096 or 8192, 2, 4 or 8);
 * wgs_per_cu: 0..16, the most workgroups of the operation's main kernel resident on one
 *             CU at a time (0 = as many as its registers and LDS allow).  A launch
 *             asks for unused dynamic LDS so that no more fit; a value at or above
 *             what the kernel reaches anyway changes nothing.  It shapes overlap
 *             (loads, decode, look-back and stores of different workgroups), not
 *             results.
 * Returns UTFX_E_INVALID_ARG for an unsupported value. */
typedef enum {
  UTFX_OP_UTF8_TO_UTF16 = 0,
  UTFX_OP_UTF16_TO_UTF8 = 1,
  UTFX_OP_VALIDATE_UTF8 = 2,
  UTFX_OP_VALIDATE_UTF16 = 3,
  UTFX_OP_LENGTH_UTF8 = 4,
  UTFX_OP_LENGTH_UTF16 = 5,
  UTFX_OP_BATCH = 6,
  UTFX_OP_COUNT_ = 7
} utfx_op;
utfx_status utfx_set_tuning(utfx_ctx *ctx, int op, uint32_t tile_bytes, uint32_t tiles_per_segment,
                            uint32_t wgs_per_cu);
utfx_status utfx_get_tuning(const utfx_ctx *ctx, int op, uint32_t *tile_bytes, uint32_t *tiles_per_segment,
                            uint32_t *wgs_per_cu);

/* ---- output-length queries (no validation) -------------------------------------- */
/* The per-unit length formula summed: UTF-16 words per UTF-8 byte = 1 for each
 * non-continuation byte plus 1 for each byte F0..FF (section 6.2: output words per
 * character); UTF-8 bytes per UTF-16 word = 1 below U+0080, 2 below U+0800, 2 for each
 * surrogate, else 3 (section 7.3).  Exact for valid input and an upper bound of what
 * the transcode stores otherwise, so cap = length is always large enough. */
utfx_result utfx_utf16_length_from_utf8(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes);
utfx_result utfx_utf8_length_from_utf16le(utfx_ctx *ctx, const uint16_t *in, size_t n_words);

/* ---- validation (section 6.4 rules 1-6; sections 2.1 and 7.4 surrogate pairing) -- */
utfx_result utfx_validate_utf8(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes);
utfx_result utfx_validate_utf16le(utfx_ctx *ctx, const uint16_t *in, size_t n_words);

/* ---- validating transcode (sections 6 and 7) ------------------------------------- */
/* out has room for cap units.  The transcode stores out[0:written] of the valid
 * prefix and may store unspecified values in out[written:cap] after an error. */
utfx_result utfx_utf8_to_utf16le(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                 uint16_t *out, size_t cap_words);
utfx_result utfx_utf16le_to_utf8(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                 uint8_t *out, size_t cap_bytes);

/* ---- asynchronous twins ----------------------------------------------------------
 * Same operations, queued on the context's stream; the result is stored to the
 * device pointer d_result when the work completes.  The return value reports only
 * argument errors and launch failures (UTFX_OK if queued).  Nothing is queued when
 * the arguments are invalid. */
utfx_status utfx_utf16_length_from_utf8_async(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                              utfx_result *d_result);
utfx_status utfx_utf8_length_from_utf16le_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                                utfx_result *d_result);
utfx_status utfx_validate_utf8_async(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                     utfx_result *d_result);
utfx_status utfx_validate_utf16le_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                        utfx_result *d_result);
utfx_status utfx_utf8_to_utf16le_async(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                       uint16_t *out, size_t cap_words, utfx_result *d_result);
utfx_status utfx_utf16le_to_utf8_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                       uint8_t *out, size_t cap_bytes, utfx_result *d_result);

/* ---- allocation-free UTF-8 -> UTF-16LE ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same operation and result as
 * utfx_utf8_to_utf16le_async, without a context: queued on hip_stream (a hipStream_t;
 * NULL = the default stream) of the current device, with the result stored to the
 * device pointer d_result.  in, out and d_result are device pointers owned by the
 * caller; out needs 2-byte alignment.
 *
 * The call allocates nothing.  Its workspace (a header and one status word per 32 KiB
 * of input, 2 MiB in all) is a static device array that each device holds until the
 * process ends; its first call on a device looks the array up and queues a kernel
 * that clears it (make that first call outside a graph capture).  Every call on a
 * device shares that device's array, so calls that overlap in time on one device (on
 * different streams or from different threads) race and give wrong results: order
 * them on one stream.  n_bytes above UTFX_NOALLOC_MAX_BYTES, a null pointer with a
 * nonzero size, a null d_result or a misaligned out give UTFX_E_INVALID_ARG with
 * nothing queued; a HIP failure gives UTFX_E_DEVICE. */
#define UTFX_NOALLOC_MAX_BYTES ((((uint64_t)1) << 29) - 32)
utfx_status utfx_utf8_to_utf16le_noalloc(const uint8_t *in, size_t n_bytes, uint16_t *out, size_t cap_words,
                                         utfx_result *d_result, void *hip_stream);

/* ---- UTF-16BE ------------------------------------------------------------------
 * The same operations with big-endian UTF-16 code units (section 2: the paper works
 * in UTF-16LE, and big-endian input or output differs only by the byte order within
 * each 16-bit unit, which the kernels swap on load or on store).
 * Arguments, results and errors are exactly those of the UTF-16LE calls above. */
utfx_result utfx_utf8_length_from_utf16be(utfx_ctx *ctx, const uint16_t *in, size_t n_words);
utfx_result utfx_validate_utf16be(utfx_ctx *ctx, const uint16_t *in, size_t n_words);
utfx_result utfx_utf8_to_utf16be(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                 uint16_t *out, size_t cap_words);
utfx_result utfx_utf16be_to_utf8(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                 uint8_t *out, size_t cap_bytes);
utfx_status utfx_utf8_length_from_utf16be_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                                utfx_result *d_result);
utfx_status utfx_validate_utf16be_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                        utfx_result *d_result);
utfx_status utfx_utf8_to_utf16be_async(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                       uint16_t *out, size_t cap_words, utfx_result *d_result);
utfx_status utfx_utf16be_to_utf8_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                       uint8_t *out, size_t cap_bytes, utfx_result *d_result);

/* ---- UTF-32LE ------------------------------------------------------------------
 * One 32-bit unit per character (section 2).  A unit in U+D800..DFFF is a
 * UTFX_E_SURROGATE error and one above U+10FFFF a UTFX_E_TOO_LARGE error, at its own
 * offset; UTF-8 input is validated exactly as by utfx_validate_utf8.  UTF-32 pointers
 * must be 4-byte aligned (else UTFX_E_INVALID_ARG); lengths are in 32-bit units.
 * Results and errors otherwise follow the UTF-16 calls: count is the offset of the
 * first invalid unit on an error, written the output units of the valid prefix.
 * Room for n_bytes units (UTF-8 -> UTF-32) or 4 n_units bytes (UTF-32 -> UTF-8)
 * always suffices. */
utfx_result utfx_validate_utf32le(utfx_ctx *ctx, const uint32_t *in, size_t n_units);
utfx_result utfx_utf8_to_utf32le(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                 uint32_t *out, size_t cap_units);
utfx_result utfx_utf32le_to_utf8(utfx_ctx *ctx, const uint32_t *in, size_t n_units,
                                 uint8_t *out, size_t cap_bytes);
utfx_status utfx_validate_utf32le_async(utfx_ctx *ctx, const uint32_t *in, size_t n_units,
                                        utfx_result *d_result);
utfx_status utfx_utf8_to_utf32le_async(utfx_ctx *ctx, const uint8_t *in, size_t n_bytes,
                                       uint32_t *out, size_t cap_units, utfx_result *d_result);
utfx_status utfx_utf32le_to_utf8_async(utfx_ctx *ctx, const uint32_t *in, size_t n_units,
                                       uint8_t *out, size_t cap_bytes, utfx_result *d_result);
/* UTF-16LE <-> UTF-32LE: UTF-16 input is validated exactly as by utfx_validate_utf16le
 * (an unpaired surrogate is UTFX_E_SURROGATE at its offset) and a pair becomes one
 * code point (section 2.1); UTF-32 input as above, a code point above U+FFFF becoming
 * a surrogate pair.  Room for n_words units (UTF-16 -> UTF-32) or 2 n_units words
 * (UTF-32 -> UTF-16) always suffices. */
utfx_result utfx_utf16le_to_utf32le(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                    uint32_t *out, size_t cap_units);
utfx_result utfx_utf32le_to_utf16le(utfx_ctx *ctx, const uint32_t *in, size_t n_units,
                                    uint16_t *out, size_t cap_words);
utfx_status utfx_utf16le_to_utf32le_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                          uint32_t *out, size_t cap_units, utfx_result *d_result);
utfx_status utfx_utf32le_to_utf16le_async(utfx_ctx *ctx, const uint32_t *in, size_t n_units,
                                          uint16_t *out, size_t cap_words, utfx_result *d_result);
/* The same with UTF-16BE words (section 2: the byte order within each 16-bit unit). */
utfx_result utfx_utf16be_to_utf32le(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                    uint32_t *out, size_t cap_units);
utfx_result utfx_utf32le_to_utf16be(utfx_ctx *ctx, const uint32_t *in, size_t n_units,
                                    uint16_t *out, size_t cap_words);
utfx_status utfx_utf16be_to_utf32le_async(utfx_ctx *ctx, const uint16_t *in, size_t n_words,
                                          uint32_t *out, size_t cap_units, utfx_result *d_result);
utfx_status utfx_utf32le_to_utf16be_async(utfx_ctx *ctx, const uint32_t *in, size_t n_units,
                                          uint16_t *out, size_t cap_words, utfx_result *d_result);

/* ---- streams: input in chunks cut at any unit offset -------------------------
 * A stream transcodes input that arrives in pieces.  Its result is the result of the
 * single-buffer call on the concatenation of all its chunks: the same output, split
 * over the calls, and the same first error at the same stream offset.  Each call
 * transcodes every character that is complete by the end of its chunk and carries
 * the unfinished one (at most 3 bytes of UTF-8, or one high surrogate of UTF-16) in
 * the stream state to the next call, so that, as in section 6, the input advances by
 * whole sequences only, and, as with the surrogate carry of section 7.4, a high
 * surrogate at the end of a chunk is paired with the first word of the next.  The
 * state lives on the host and holds no device memory. */
typedef enum {
  UTFX_STREAM_UTF8_TO_UTF16LE = 0,
  UTFX_STREAM_UTF16LE_TO_UTF8 = 1,
  UTFX_STREAM_UTF8_TO_UTF16BE = 2,
  UTFX_STREAM_UTF16BE_TO_UTF8 = 3
} utfx_stream_format;

typedef struct {
  uint64_t in_units;   /* input units passed in so far (carried units included) */
  uint64_t out_units;  /* output units written so far */
  uint64_t err_offset; /* stream offset of the encoding error that ended the stream */
  int32_t format;      /* utfx_stream_format */
  int32_t status;      /* UTFX_OK, or that encoding error */
  uint32_t n_carry;    /* units carried into the next call: 0..3 bytes, or 0..1 word */
  uint32_t finished;   /* 1 after a successful call with final != 0 */
  uint8_t carry[4];    /* the carried units as they were in memory */
  uint8_t carry_need;  /* units the carried character still needs */
  uint8_t carry_out;   /* output units it makes once complete and valid */
  uint16_t reserved;
} utfx_stream;

/* Starts a stream (any previous state is discarded).  UTFX_E_INVALID_ARG for a null
 * state or an unknown format.  Host only: launches nothing. */
utfx_status utfx_stream_init(utfx_stream *st, int format);

/* Passes the next chunk: in (device; UTF-16 2-byte aligned) holds n_units input
 * units, out (device; UTF-16 2-byte aligned) has room for cap_units output units.
 * final != 0 marks the last chunk: a character left unfinished there is an error
 * (UTFX_E_MISSING_CONT, or UTFX_E_SURROGATE for a high surrogate) instead of being
 * carried.  Room for (n_carry + n_units) units of output (UTF-16 out), or three times
 * that (UTF-8 out), always suffices.  Synchronous: it blocks until the result is on
 * the host; not allowed during graph capture.
 *   OK:               count = written = output units stored by this call in
 *                     out[0:written]; the state advances (in_units += n_units).
 *   encoding error:   count = offset of the first invalid unit in the whole stream
 *                     (stream offsets start at 0 with the first chunk's first unit);
 *                     written = output units of the valid characters before it that
 *                     this call produced, in out[0:min(written, cap)].  The stream is
 *                     then over: later calls return the same status and offset with
 *                     written = 0 until utfx_stream_init.
 *   OUTPUT_TOO_SMALL: count = output units this call needs, written = 0; the state
 *                     does not change, so the same chunk can be passed again with a
 *                     larger buffer.
 *   INVALID_ARG:      null or malformed state, bad pointers, or a call after the
 *                     final chunk; the state does not change.
 * Output beyond `written` is unspecified; nothing is stored at or beyond cap. */
utfx_result utfx_stream_transcode(utfx_ctx *ctx, utfx_stream *st, const void *in, size_t n_units,
                                  void *out, size_t cap_units, int final);

/* ---- batched: many independent strings in one call ---------------------------- */
/* One string.  in_off/out_off are byte offsets into the arenas; in_len is in input
 * units and out_cap in output units; dir 0 = UTF-8 -> UTF-16LE, 1 = UTF-16LE -> UTF-8.
 * UTF-16 data (the input of dir 1, the output of dir 0) must start at an even
 * address.  Each item gets the same result as the single-buffer call on its bytes;
 * an item with a bad descriptor (dir > 1, odd UTF-16 address, in_len above
 * UTFX_MAX_UNITS, input or output slot not inside its arena) gets
 * UTFX_E_INVALID_ARG.  Items may share input; their outputs must not overlap. */
typedef struct {
  uint64_t in_off;
  uint64_t in_len;
  uint64_t out_off;
  uint64_t out_cap;
  uint32_t dir;
  uint32_t pad;
} utfx_item;

/* Runs the batch: the arenas hold in_bytes and out_bytes bytes; d_items (device,
 * n_items entries) describe the strings, d_results (device, n_items entries) receive
 * one result each.  Strings of up to 16,384 units (the wave_max_units tunable below)
 * are transcoded by one wavefront each; longer ones are cut into segments, one
 * workgroup each, with a look-back that ends at the string's first segment (sections 6
 * and 7 per string).  The plan is built on the device, so
 * the call issues a fixed sequence of kernels with no allocation and no host
 * synchronisation once the workspace is large enough: it can be captured into a HIP
 * graph and replayed with new contents of the same buffers.  total_in_units bounds
 * the sum of in_len over the items (it sizes the plan); if the items add up to more,
 * every string above 16,384 units gets UTFX_E_INVALID_ARG.  Growing the workspace
 * (first call, or a larger n_items / total_in_units) synchronises the stream once.
 * Returns UTFX_OK if queued, UTFX_E_INVALID_ARG for null pointers. */
utfx_status utfx_batch_run(utfx_ctx *ctx, const uint8_t *in_arena, size_t in_bytes, uint8_t *out_arena,
                           size_t out_bytes, const utfx_item *d_items, uint32_t n_items,
                           uint64_t total_in_units, utfx_result *d_results);
/* Tunables of the batched call, picked by the autotuner (they shape the schedule, never
 * the results): wave_max_units (1024 .. 262144, default 16384): strings of at most this
 * many units are walked by one wavefront, longer ones take segments;
 * large_tiles_per_segment (2 or 4, default 4): a segment is that many 8 KiB tiles of
 * UTF-8 (4096 words of UTF-16); large_wgs_per_cu (1 or 2, default 2): persistent
 * segment workgroups launched per CU.  The "more than 16,384 units" above reads "more
 * than wave_max_units".  UTFX_E_INVALID_ARG for other values. */
utfx_status utfx_set_batch_tuning(utfx_ctx *ctx, uint32_t wave_max_units, uint32_t large_tiles_per_segment,
                                  uint32_t large_wgs_per_cu);
utfx_status utfx_get_batch_tuning(const utfx_ctx *ctx, uint32_t *wave_max_units,
                                  uint32_t *large_tiles_per_segment, uint32_t *large_wgs_per_cu);

/* ---- HIP graphs: record a sequence of calls once, replay it many times ---------- */
/* Between utfx_capture_begin and utfx_capture_end, the context's _async calls and
 * utfx_batch_run are recorded into a HIP graph instead of being run (on a private
 * capture stream).  Every kernel takes its description from its arguments and from
 * device memory, and no call records a memset, so a replay runs the same calls on the
 * buffers' contents at replay time: refill inputs or item tables between replays,
 * keep sizes and pointers.  Calls that would allocate or synchronise are refused
 * while capturing (UTFX_E_INVALID_ARG): synchronous calls, and calls whose workspace
 * would have to grow -- make each call once eagerly first.  Launch a graph on any
 * stream; replays of graphs made on one context must not overlap in time.  One graph
 * per capture; utfx_graph_destroy frees it (the context must outlive its graphs).
 * A graph holds the addresses of the context's workspace: once an eager call on the
 * context has grown (reallocated) the workspace, utfx_graph_launch refuses that graph
 * with UTFX_E_INVALID_ARG instead of replaying kernels on freed memory; capture it
 * again. */
typedef struct utfx_graph utfx_graph;
utfx_status utfx_capture_begin(utfx_ctx *ctx);
utfx_status utfx_capture_end(utfx_ctx *ctx, utfx_graph **graph);
utfx_status utfx_graph_launch(utfx_graph *graph, void *hip_stream);
void utfx_graph_destroy(utfx_graph *graph);

/* ---- serving: continuous batching of host requests ------------------------------ */
/* A server owns `inflight` slots, each with its own HIP stream, context, device
 * arenas and pinned host staging.  Submitted requests (host payloads) wait in a
 * queue.  Whenever a slot is free, utfx_server_progress packs every queued request
 * that fits the slot's arenas and item count (admission by free arena bytes, in
 * arrival order) into one step: host-to-device copy, one utfx_batch_run, device-to-
 * host copy of results and outputs.  Requests arriving meanwhile join the next step
 * (continuous batching); with inflight >= 2, steps overlap.  Requests of 1 MiB of input
 * or more are batched apart from smaller ones, in steps of their own with one such
 * step in flight while smaller requests wait, so that those do not wait behind large
 * transfers.  When a step completes,
 * each request's output (its valid prefix, `written` units) is in its `out` buffer
 * and a completion {tag, result} is reported.  Requests of 64 KiB or more whose
 * payload or output buffer is pinned host memory skip the staging copy: that data
 * moves by DMA straight between the buffer and the device (a direct output is copied
 * whole, so out[written:out_cap] then holds unspecified values).  A request larger than an arena
 * completes with UTFX_E_INVALID_ARG; the requests of a step that could not be launched
 * (a failed copy or batched call) complete with UTFX_E_DEVICE and
 * utfx_server_last_error() holds the reason.  Payloads and outputs must stay valid until the
 * request completes.  Single-threaded: one thread drives a server. */
typedef struct utfx_server utfx_server;
typedef struct {
  uint64_t arena_in_bytes;   /* input arena bytes per slot */
  uint64_t arena_out_bytes;  /* output arena bytes per slot */
  uint64_t device_cap_bytes; /* limit on inflight * (in + out) device bytes; 0 = none */
  uint32_t max_items;        /* requests per step (1 = one launch per request) */
  uint32_t inflight;         /* slots, 1..16 */
} utfx_server_config;
typedef struct {
  uint64_t tag;
  utfx_result result;
} utfx_completion;
utfx_status utfx_server_create(utfx_server **srv, const utfx_server_config *cfg);
void utfx_server_destroy(utfx_server *srv);
const char *utfx_server_last_error(const utfx_server *srv);
/* Queues one request: len_units input units at host address data, direction dir
 * (0 = UTF-8 -> UTF-16LE, 1 = UTF-16LE -> UTF-8), output to host address out with room
 * for out_cap_units output units.  With UTFX_SERVER_DEVICE_BUFFERS or-ed into dir, data
 * and out are device addresses instead (a device-resident request): a kernel on the
 * slot's stream gathers the payload into the step's input arena and another copies the
 * valid prefix of the output (`written` units, at most out_cap_units) to out, so only
 * the 24-byte result crosses PCIe. */
#define UTFX_SERVER_DEVICE_BUFFERS 0x100u
utfx_status utfx_server_submit(utfx_server *srv, uint64_t tag, const void *data, uint64_t len_units,
                               uint32_t dir, void *out, uint64_t out_cap_units);
/* Reports up to max_done completions (drains a slot only when all its requests fit)
 * and launches steps on free slots.  Never blocks. */
utfx_status utfx_server_progress(utfx_server *srv, utfx_completion *done, uint32_t max_done,
                                 uint32_t *n_done);
/* Replays an arrival trace in real time: request i (tag i) is submitted once
 * arrival_ns[i] (ascending, from the call's start) has passed, and progress runs
 * continuously until all n complete.  latency_ns[i] = completion - arrival (result and
 * output on the host); results[i] its result; *wall_ns the replay's duration. */
utfx_status utfx_server_replay(utfx_server *srv, uint32_t n, const uint64_t *arrival_ns,
                               const void *const *data, const uint64_t *len_units, const uint32_t *dirs,
                               void *const *outs, const uint64_t *out_caps, uint64_t *latency_ns,
                               utfx_result *results, uint64_t *wall_ns);

#ifdef __cplusplus
}
#endif
#endif /* UTFX_H */
