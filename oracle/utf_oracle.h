/*
 * utf_oracle.h -- scalar CPU oracle for validating UTF-8 <-> UTF-16LE transcoding.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library; the status codes below are
 * a separate copy, and a test asserts that both copies agree.
 *
 * What it computes (Clausecker & Lemire, "Transcoding Unicode Characters with
 * AVX-512 Instructions"):
 *   - the code-point space and the UTF-16 surrogate mechanism of section 2.1;
 *   - the UTF-8 byte types of Table 1 and the shortest-form / range rules of
 *     section 2.2, restated as the six validation rules of section 6.4;
 *   - the bit correspondence of Figure 1(a);
 *   - the abort semantics of sections 6.4 and 7.4: on the first encoding error the
 *     characters before it are transcoded and the call ends, reporting where.
 *
 * Result convention (shared by every entry point):
 *   status  UTFX_REF_OK or one of the error kinds below
 *   count   OK: units produced (transcode), n (validate), length (length query);
 *           encoding error: offset, in input code units, of the first invalid unit;
 *           OUTPUT_TOO_SMALL: output units the input needs
 *   written transcode: output units of the valid prefix in[0:count] (on OK equal to
 *           count; on OUTPUT_TOO_SMALL 0).  validate and length: equal to count.
 * Only out[0 : min(written, cap)] is defined after a transcode; nothing is ever
 * stored at or beyond cap.
 */
#ifndef UTF_ORACLE_H
#define UTF_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  UTFX_REF_OK = 0,
  UTFX_REF_E_STRAY_CONT = 1,      /* UTF-8: continuation byte where a character must start (rule 3) */
  UTFX_REF_E_MISSING_CONT = 2,    /* UTF-8: lead byte without its continuation bytes (rule 2) */
  UTFX_REF_E_OVERLONG = 3,        /* UTF-8: C0/C1, or a 3/4-byte form below its minimum (rule 4) */
  UTFX_REF_E_TOO_LARGE = 4,       /* UTF-8: F4 form above U+10FFFF (rule 5) */
  UTFX_REF_E_SURROGATE = 5,       /* UTF-8: encoded U+D800..DFFF (rule 6); UTF-16: unpaired surrogate */
  UTFX_REF_E_BAD_BYTE = 6,        /* UTF-8: byte F5..FF (rule 1) */
  UTFX_REF_E_OUTPUT_TOO_SMALL = 16,
  UTFX_REF_E_INVALID_ARG = 17
};

typedef struct {
  int32_t status;
  uint32_t reserved;
  uint64_t count;
  uint64_t written;
} utfx_ref_result;

/* Output-length queries: the per-unit length formula summed, with no validation. */
utfx_ref_result utfx_ref_utf16_length_from_utf8(const uint8_t *in, size_t n_bytes);
utfx_ref_result utfx_ref_utf8_length_from_utf16le(const uint16_t *in, size_t n_words);

/* Validation only. */
utfx_ref_result utfx_ref_validate_utf8(const uint8_t *in, size_t n_bytes);
utfx_ref_result utfx_ref_validate_utf16le(const uint16_t *in, size_t n_words);

/* Validating transcode.  out may be NULL only when cap is 0. */
utfx_ref_result utfx_ref_utf8_to_utf16le(const uint8_t *in, size_t n_bytes,
                                         uint16_t *out, size_t cap_words);
utfx_ref_result utfx_ref_utf16le_to_utf8(const uint16_t *in, size_t n_words,
                                         uint8_t *out, size_t cap_bytes);

/* UTF-32LE (section 2: one 32-bit unit per character): a unit in U+D800..DFFF is a
 * SURROGATE error, one above U+10FFFF a TOO_LARGE error, at its own offset. */
utfx_ref_result utfx_ref_validate_utf32le(const uint32_t *in, size_t n_units);
utfx_ref_result utfx_ref_utf8_to_utf32le(const uint8_t *in, size_t n_bytes,
                                         uint32_t *out, size_t cap_units);
utfx_ref_result utfx_ref_utf32le_to_utf8(const uint32_t *in, size_t n_units,
                                         uint8_t *out, size_t cap_bytes);
utfx_ref_result utfx_ref_utf16le_to_utf32le(const uint16_t *in, size_t n_words,
                                            uint32_t *out, size_t cap_units);
utfx_ref_result utfx_ref_utf32le_to_utf16le(const uint32_t *in, size_t n_units,
                                            uint16_t *out, size_t cap_words);

/* Convenience loop for exhaustive tests: validates n_strings strings of len bytes
 * each, stored back to back in buf; per-string status and count go to the arrays
 * (either may be NULL).  Returns the number of valid strings. */
uint64_t utfx_ref_validate_utf8_fixed(const uint8_t *buf, size_t n_strings, size_t len,
                                      int32_t *status, uint64_t *count);
uint64_t utfx_ref_validate_utf16le_fixed(const uint16_t *buf, size_t n_strings, size_t len,
                                         int32_t *status, uint64_t *count);
/* The same loop over the validating transcodes (output room: len words, or 3 len
 * bytes, per string, discarded): per-string status, count and written. */
uint64_t utfx_ref_utf8_to_utf16le_fixed(const uint8_t *buf, size_t n_strings, size_t len,
                                        int32_t *status, uint64_t *count, uint64_t *written);
uint64_t utfx_ref_utf16le_to_utf8_fixed(const uint16_t *buf, size_t n_strings, size_t len,
                                        int32_t *status, uint64_t *count, uint64_t *written);

/* Batched reference (the invariant a batched call must meet: each string gets the
 * result of the single-string call on its bytes).  One item per string, with byte
 * offsets into the arenas, the input length in input units, the output room in output
 * units and the direction: 0 = UTF-8 -> UTF-16LE, 1 = UTF-16LE -> UTF-8.  An item whose
 * direction is above 1, whose UTF-16 side starts at an odd offset, or whose input or
 * output slot is not inside its arena gets UTFX_REF_E_INVALID_ARG.  Otherwise results[i]
 * is the single-string transcode of the item and its output is stored at out_off.
 * Returns the number of items with status OK. */
typedef struct {
  uint64_t in_off;
  uint64_t in_len;
  uint64_t out_off;
  uint64_t out_cap;
  uint32_t dir;
  uint32_t pad;
} utfx_ref_item;
uint64_t utfx_ref_batch(const uint8_t *in_arena, size_t in_bytes, uint8_t *out_arena, size_t out_bytes,
                        const utfx_ref_item *items, size_t n_items, utfx_ref_result *results);

#ifdef __cplusplus
}
#endif
#endif
