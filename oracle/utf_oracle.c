/*
 * utf_oracle.c -- scalar CPU oracle (TEST INFRASTRUCTURE ONLY; see utf_oracle.h).
 *
 * One character at a time, straight from the definitions the paper restates:
 *   section 2.1  UTF-16: BMP code points stand for themselves; others have 0x10000
 *                subtracted, the 20-bit rest split 10/10 and tagged 0xD800 / 0xDC00;
 *                a high surrogate must be followed by a low one and vice versa.
 *   section 2.2 + Table 1  UTF-8 byte types; shortest form only; nothing above
 *                U+10FFFF; C0, C1, F5..FF never appear.
 *   Figure 1(a)  which code-point bits go into which UTF-8 byte.
 *   section 2    UTF-32: each character is one 32-bit integer, its code point; the
 *                code-point space ends at U+10FFFF and U+D800..DFFF are surrogates,
 *                not characters.
 *   section 6.4  the six validation rules; on an error the characters before it are
 *                transcoded and the call stops (sections 6.4 and 7.4).
 *
 * Where the paper is silent the readings are:
 *   - error kind = the first rule the scalar decoder trips over at the offending
 *     offset, checked in this order: byte type, continuation bytes present, shortest
 *     form, surrogate range, U+10FFFF bound (the paper reports positions only);
 *   - the end of the input behaves as if padded with NUL (sections 6.3 and 7.5), so
 *     a truncated sequence is an error at its lead byte / high surrogate;
 *   - a byte-order mark and noncharacters are ordinary characters (section 2.1);
 *   - an encoding error outranks an output buffer that is too small.
 */
#include "utf_oracle.h"

static utfx_ref_result mk(int32_t status, uint64_t count, uint64_t written) {
  utfx_ref_result r;
  r.status = status;
  r.reserved = 0;
  r.count = count;
  r.written = written;
  return r;
}

/* Table 1: is b a continuation byte (10xxxxxx)? */
static int is_cont(uint8_t b) { return b >= 0x80 && b <= 0xBF; }

/* Decode the character starting at in[i].  On success returns 0 and sets *cp and
 * *len; on failure returns the error kind.  Rule numbers are those of section 6.4. */
static int32_t decode_utf8_at(const uint8_t *in, size_t n, size_t i, uint32_t *cp, size_t *len) {
  uint8_t b0 = in[i];
  uint32_t v;
  size_t k; /* number of continuation bytes */
  if (b0 <= 0x7F) {
    *cp = b0;
    *len = 1;
    return UTFX_REF_OK;
  } else if (b0 <= 0xBF) {
    return UTFX_REF_E_STRAY_CONT; /* rule 3 */
  } else if (b0 <= 0xC1) {
    return UTFX_REF_E_OVERLONG; /* C0/C1 always encode below U+0080: rule 4 */
  } else if (b0 <= 0xDF) {
    k = 1;
    v = b0 & 0x1F;
  } else if (b0 <= 0xEF) {
    k = 2;
    v = b0 & 0x0F;
  } else if (b0 <= 0xF4) {
    k = 3;
    v = b0 & 0x07;
  } else {
    return UTFX_REF_E_BAD_BYTE; /* rule 1 */
  }
  for (size_t j = 1; j <= k; j++) {
    if (i + j >= n || !is_cont(in[i + j])) return UTFX_REF_E_MISSING_CONT; /* rule 2 */
    v = (v << 6) | (uint32_t)(in[i + j] & 0x3F);
  }
  /* rule 4: shortest form -- 2-byte forms reach here only from C2..DF (>= U+0080) */
  if (k == 2 && v < 0x800) return UTFX_REF_E_OVERLONG;
  if (k == 3 && v < 0x10000) return UTFX_REF_E_OVERLONG;
  if (v >= 0xD800 && v <= 0xDFFF) return UTFX_REF_E_SURROGATE; /* rule 6 */
  if (v > 0x10FFFF) return UTFX_REF_E_TOO_LARGE;                /* rule 5 */
  *cp = v;
  *len = k + 1;
  return UTFX_REF_OK;
}

/* Section 2.1: decode the character starting at in[i] of a UTF-16LE string. */
static int32_t decode_utf16_at(const uint16_t *in, size_t n, size_t i, uint32_t *cp, size_t *len) {
  uint16_t w = in[i];
  if (w >= 0xD800 && w <= 0xDBFF) {
    if (i + 1 >= n) return UTFX_REF_E_SURROGATE;
    uint16_t lo = in[i + 1];
    if (lo < 0xDC00 || lo > 0xDFFF) return UTFX_REF_E_SURROGATE;
    *cp = 0x10000u + (((uint32_t)(w - 0xD800) << 10) | (uint32_t)(lo - 0xDC00));
    *len = 2;
    return UTFX_REF_OK;
  }
  if (w >= 0xDC00 && w <= 0xDFFF) return UTFX_REF_E_SURROGATE;
  *cp = w;
  *len = 1;
  return UTFX_REF_OK;
}

/* Section 2: a UTF-32 unit is a character if it is a code point (at most 0x10FFFF)
 * outside the surrogate range. */
static int32_t decode_utf32_at(const uint32_t *in, size_t i, uint32_t *cp) {
  uint32_t u = in[i];
  if (u >= 0xD800 && u <= 0xDFFF) return UTFX_REF_E_SURROGATE;
  if (u > 0x10FFFF) return UTFX_REF_E_TOO_LARGE;
  *cp = u;
  return UTFX_REF_OK;
}

/* Section 2.1: the UTF-16 form of a scalar value; returns the number of words. */
static size_t encode_utf16(uint32_t cp, uint16_t w[2]) {
  if (cp < 0x10000) {
    w[0] = (uint16_t)cp;
    return 1;
  }
  uint32_t v = cp - 0x10000;
  w[0] = (uint16_t)(0xD800 + (v >> 10));
  w[1] = (uint16_t)(0xDC00 + (v & 0x3FF));
  return 2;
}

/* Figure 1(a): the UTF-8 form of a scalar value; returns the number of bytes. */
static size_t encode_utf8(uint32_t cp, uint8_t b[4]) {
  if (cp < 0x80) {
    b[0] = (uint8_t)cp;
    return 1;
  }
  if (cp < 0x800) {
    b[0] = (uint8_t)(0xC0 | (cp >> 6));
    b[1] = (uint8_t)(0x80 | (cp & 0x3F));
    return 2;
  }
  if (cp < 0x10000) {
    b[0] = (uint8_t)(0xE0 | (cp >> 12));
    b[1] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
    b[2] = (uint8_t)(0x80 | (cp & 0x3F));
    return 3;
  }
  b[0] = (uint8_t)(0xF0 | (cp >> 18));
  b[1] = (uint8_t)(0x80 | ((cp >> 12) & 0x3F));
  b[2] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
  b[3] = (uint8_t)(0x80 | (cp & 0x3F));
  return 4;
}

/* ---- length queries: a per-unit formula, summed; no validation ---------------- */

/* UTF-16 words produced per UTF-8 byte: one per non-continuation byte, plus one more
 * for every 4-byte lead (whose character needs a surrogate pair). */
utfx_ref_result utfx_ref_utf16_length_from_utf8(const uint8_t *in, size_t n) {
  if (n > 0 && in == 0) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  uint64_t total = 0;
  for (size_t i = 0; i < n; i++) {
    if (!is_cont(in[i])) total += 1;
    if (in[i] >= 0xF0) total += 1;
  }
  return mk(UTFX_REF_OK, total, total);
}

/* UTF-8 bytes produced per UTF-16 word: 1 below U+0080, 2 below U+0800, 2 for each
 * half of a surrogate pair (4 bytes per pair), else 3. */
utfx_ref_result utfx_ref_utf8_length_from_utf16le(const uint16_t *in, size_t n) {
  if (n > 0 && in == 0) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  uint64_t total = 0;
  for (size_t i = 0; i < n; i++) {
    uint16_t w = in[i];
    if (w < 0x80)
      total += 1;
    else if (w < 0x800)
      total += 2;
    else if (w >= 0xD800 && w <= 0xDFFF)
      total += 2;
    else
      total += 3;
  }
  return mk(UTFX_REF_OK, total, total);
}

/* ---- validation ---------------------------------------------------------------- */

utfx_ref_result utfx_ref_validate_utf8(const uint8_t *in, size_t n) {
  if (n > 0 && in == 0) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  size_t i = 0;
  while (i < n) {
    uint32_t cp;
    size_t len;
    int32_t st = decode_utf8_at(in, n, i, &cp, &len);
    if (st != UTFX_REF_OK) return mk(st, i, i);
    i += len;
  }
  return mk(UTFX_REF_OK, n, n);
}

utfx_ref_result utfx_ref_validate_utf16le(const uint16_t *in, size_t n) {
  if (n > 0 && in == 0) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  size_t i = 0;
  while (i < n) {
    uint32_t cp;
    size_t len;
    int32_t st = decode_utf16_at(in, n, i, &cp, &len);
    if (st != UTFX_REF_OK) return mk(st, i, i);
    i += len;
  }
  return mk(UTFX_REF_OK, n, n);
}

utfx_ref_result utfx_ref_validate_utf32le(const uint32_t *in, size_t n) {
  if (n > 0 && in == 0) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  for (size_t i = 0; i < n; i++) {
    uint32_t cp;
    int32_t st = decode_utf32_at(in, i, &cp);
    if (st != UTFX_REF_OK) return mk(st, i, i);
  }
  return mk(UTFX_REF_OK, n, n);
}

/* ---- validating transcode ------------------------------------------------------ */

utfx_ref_result utfx_ref_utf8_to_utf16le(const uint8_t *in, size_t n, uint16_t *out, size_t cap) {
  if ((n > 0 && in == 0) || (cap > 0 && out == 0)) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  size_t i = 0;
  uint64_t o = 0;
  while (i < n) {
    uint32_t cp;
    size_t len;
    int32_t st = decode_utf8_at(in, n, i, &cp, &len);
    if (st != UTFX_REF_OK) return mk(st, i, o);
    uint16_t w[2];
    size_t k = encode_utf16(cp, w);
    for (size_t j = 0; j < k; j++) {
      if (o < cap) out[o] = w[j];
      o++;
    }
    i += len;
  }
  if (o > cap) return mk(UTFX_REF_E_OUTPUT_TOO_SMALL, o, 0);
  return mk(UTFX_REF_OK, o, o);
}

utfx_ref_result utfx_ref_utf16le_to_utf8(const uint16_t *in, size_t n, uint8_t *out, size_t cap) {
  if ((n > 0 && in == 0) || (cap > 0 && out == 0)) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  size_t i = 0;
  uint64_t o = 0;
  while (i < n) {
    uint32_t cp;
    size_t len;
    int32_t st = decode_utf16_at(in, n, i, &cp, &len);
    if (st != UTFX_REF_OK) return mk(st, i, o);
    uint8_t b[4];
    size_t k = encode_utf8(cp, b);
    for (size_t j = 0; j < k; j++) {
      if (o < cap) out[o] = b[j];
      o++;
    }
    i += len;
  }
  if (o > cap) return mk(UTFX_REF_E_OUTPUT_TOO_SMALL, o, 0);
  return mk(UTFX_REF_OK, o, o);
}

utfx_ref_result utfx_ref_utf8_to_utf32le(const uint8_t *in, size_t n, uint32_t *out, size_t cap) {
  if ((n > 0 && in == 0) || (cap > 0 && out == 0)) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  size_t i = 0;
  uint64_t o = 0;
  while (i < n) {
    uint32_t cp;
    size_t len;
    int32_t st = decode_utf8_at(in, n, i, &cp, &len);
    if (st != UTFX_REF_OK) return mk(st, i, o);
    if (o < cap) out[o] = cp;
    o++;
    i += len;
  }
  if (o > cap) return mk(UTFX_REF_E_OUTPUT_TOO_SMALL, o, 0);
  return mk(UTFX_REF_OK, o, o);
}

utfx_ref_result utfx_ref_utf32le_to_utf8(const uint32_t *in, size_t n, uint8_t *out, size_t cap) {
  if ((n > 0 && in == 0) || (cap > 0 && out == 0)) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  uint64_t o = 0;
  for (size_t i = 0; i < n; i++) {
    uint32_t cp;
    int32_t st = decode_utf32_at(in, i, &cp);
    if (st != UTFX_REF_OK) return mk(st, i, o);
    uint8_t b[4];
    size_t k = encode_utf8(cp, b);
    for (size_t j = 0; j < k; j++) {
      if (o < cap) out[o] = b[j];
      o++;
    }
  }
  if (o > cap) return mk(UTFX_REF_E_OUTPUT_TOO_SMALL, o, 0);
  return mk(UTFX_REF_OK, o, o);
}

utfx_ref_result utfx_ref_utf16le_to_utf32le(const uint16_t *in, size_t n, uint32_t *out, size_t cap) {
  if ((n > 0 && in == 0) || (cap > 0 && out == 0)) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  size_t i = 0;
  uint64_t o = 0;
  while (i < n) {
    uint32_t cp;
    size_t len;
    int32_t st = decode_utf16_at(in, n, i, &cp, &len);
    if (st != UTFX_REF_OK) return mk(st, i, o);
    if (o < cap) out[o] = cp;
    o++;
    i += len;
  }
  if (o > cap) return mk(UTFX_REF_E_OUTPUT_TOO_SMALL, o, 0);
  return mk(UTFX_REF_OK, o, o);
}

utfx_ref_result utfx_ref_utf32le_to_utf16le(const uint32_t *in, size_t n, uint16_t *out, size_t cap) {
  if ((n > 0 && in == 0) || (cap > 0 && out == 0)) return mk(UTFX_REF_E_INVALID_ARG, 0, 0);
  uint64_t o = 0;
  for (size_t i = 0; i < n; i++) {
    uint32_t cp;
    int32_t st = decode_utf32_at(in, i, &cp);
    if (st != UTFX_REF_OK) return mk(st, i, o);
    uint16_t w[2];
    size_t k = encode_utf16(cp, w);
    for (size_t j = 0; j < k; j++) {
      if (o < cap) out[o] = w[j];
      o++;
    }
  }
  if (o > cap) return mk(UTFX_REF_E_OUTPUT_TOO_SMALL, o, 0);
  return mk(UTFX_REF_OK, o, o);
}

/* ---- loops for exhaustive tests ------------------------------------------------ */

uint64_t utfx_ref_validate_utf8_fixed(const uint8_t *buf, size_t n_strings, size_t len,
                                      int32_t *status, uint64_t *count) {
  uint64_t valid = 0;
  for (size_t s = 0; s < n_strings; s++) {
    utfx_ref_result r = utfx_ref_validate_utf8(buf + s * len, len);
    if (status) status[s] = r.status;
    if (count) count[s] = r.count;
    if (r.status == UTFX_REF_OK) valid++;
  }
  return valid;
}

uint64_t utfx_ref_validate_utf16le_fixed(const uint16_t *buf, size_t n_strings, size_t len,
                                         int32_t *status, uint64_t *count) {
  uint64_t valid = 0;
  for (size_t s = 0; s < n_strings; s++) {
    utfx_ref_result r = utfx_ref_validate_utf16le(buf + s * len, len);
    if (status) status[s] = r.status;
    if (count) count[s] = r.count;
    if (r.status == UTFX_REF_OK) valid++;
  }
  return valid;
}

uint64_t utfx_ref_utf8_to_utf16le_fixed(const uint8_t *buf, size_t n_strings, size_t len,
                                        int32_t *status, uint64_t *count, uint64_t *written) {
  uint64_t valid = 0;
  uint16_t out[64];
  if (len > 64) return 0;
  for (size_t s = 0; s < n_strings; s++) {
    utfx_ref_result r = utfx_ref_utf8_to_utf16le(buf + s * len, len, out, len);
    if (status) status[s] = r.status;
    if (count) count[s] = r.count;
    if (written) written[s] = r.written;
    if (r.status == UTFX_REF_OK) valid++;
  }
  return valid;
}

uint64_t utfx_ref_utf16le_to_utf8_fixed(const uint16_t *buf, size_t n_strings, size_t len,
                                        int32_t *status, uint64_t *count, uint64_t *written) {
  uint64_t valid = 0;
  uint8_t out[192];
  if (len > 64) return 0;
  for (size_t s = 0; s < n_strings; s++) {
    utfx_ref_result r = utfx_ref_utf16le_to_utf8(buf + s * len, len, out, 3 * len);
    if (status) status[s] = r.status;
    if (count) count[s] = r.count;
    if (written) written[s] = r.written;
    if (r.status == UTFX_REF_OK) valid++;
  }
  return valid;
}

/* ---- batched reference: every item is the single-string call on its bytes ------- */

uint64_t utfx_ref_batch(const uint8_t *in_arena, size_t in_bytes, uint8_t *out_arena, size_t out_bytes,
                        const utfx_ref_item *items, size_t n_items, utfx_ref_result *results) {
  uint64_t ok = 0;
  for (size_t i = 0; i < n_items; i++) {
    const utfx_ref_item it = items[i];
    const uint64_t in_unit = it.dir == 1 ? 2 : 1, out_unit = it.dir == 1 ? 1 : 2;
    int bad = it.dir > 1;
    if (!bad) bad = it.in_off > in_bytes || it.in_len > (in_bytes - it.in_off) / in_unit;
    if (!bad) bad = it.out_off > out_bytes || it.out_cap > (out_bytes - it.out_off) / out_unit;
    if (!bad) bad = (it.dir == 1 && (it.in_off & 1)) || (it.dir == 0 && (it.out_off & 1));
    if (bad) {
      results[i] = mk(UTFX_REF_E_INVALID_ARG, 0, 0);
      continue;
    }
    if (it.dir == 0)
      results[i] = utfx_ref_utf8_to_utf16le(in_arena + it.in_off, it.in_len,
                                            (uint16_t *)(void *)(out_arena + it.out_off), it.out_cap);
    else
      results[i] = utfx_ref_utf16le_to_utf8((const uint16_t *)(const void *)(in_arena + it.in_off), it.in_len,
                                            out_arena + it.out_off, it.out_cap);
    if (results[i].status == UTFX_REF_OK) ok++;
  }
  return ok;
}
