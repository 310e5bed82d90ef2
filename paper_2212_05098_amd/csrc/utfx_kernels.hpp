// utfx_kernels.hpp -- gfx950 building blocks and the length / validate kernels for
// validating UTF-8 <-> UTF-16LE transcoding (the transcode kernels that use these
// blocks are in utfx_transcode.hpp).
//
// One kernel family per operation: output-length query (reduction), validate
// (first-error minimum) and transcode (one look-back per segment + LDS-staged
// coalesced stores), each followed by a one-workgroup finalisation kernel.  What is
// computed follows Clausecker & Lemire: the UTF-8 byte classes of Table 1, the six
// validation rules of section 6.4, the bit layout of Figure 1(a), the surrogate
// arithmetic of sections 6.2 and 7.2, and the abort-at-first-error contract of
// sections 6.4 and 7.4.  How it is computed is GPU-specific:
//   * a workgroup owns a segment of `seg` tiles; a tile is one 16-byte chunk per
//     thread, classified SWAR-style (four bytes per 32-bit operation);
//   * the paper's serial "advance by the bytes consumed" chain becomes, per segment,
//     a cheap counting pass (the per-byte output-length formula), one decoupled
//     look-back across segments, and a per-tile workgroup scan; the segment is read
//     twice, the second time from cache;
//   * the paper's compress instruction becomes a scatter into LDS followed by
//     coalesced 16-byte stores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "utfx_device.hpp"

namespace utfx_dev {

// ================================================================ UTF-8 loading

// 16 bytes at grid position q0 (aligned).  Bytes outside the input read as 0 (NUL),
// the padding convention of section 6.3: a NUL is not a continuation byte, so a
// truncated sequence at the end fails like any other missing continuation.
__device__ __forceinline__ void load8(const Launch& L, uint64_t q0, uint32_t x[4]) {
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  if (q0 >= lo && q0 + 16 <= hi) {
    uint4 v = *reinterpret_cast<const uint4*>(L.base + q0);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else {
    x[0] = x[1] = x[2] = x[3] = 0;
    if (q0 + 16 <= lo || q0 >= hi) return;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      uint64_t q = q0 + i;
      if (q >= lo && q < hi) x[i >> 2] |= (uint32_t)L.base[q] << (8 * (i & 3));
    }
  }
}

// The 4 bytes before grid position q0 (q0 is a multiple of 16).
__device__ __forceinline__ uint32_t load8_prev(const Launch& L, uint64_t q0) {
  if (q0 == 0) return 0;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const uint64_t q = q0 - 4;
  if (q >= lo && q + 4 <= hi) return *reinterpret_cast<const uint32_t*>(L.base + q);
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (q + i >= lo && q + i < hi) r |= (uint32_t)L.base[q + i] << (8 * i);
  }
  return r;
}

// Byte masks (0xFF per byte) of the chunk bytes a <= i < b (0 <= a, b <= 16).
__device__ __forceinline__ void byte_masks_ab(uint32_t a, uint32_t b, uint32_t m[4]) {
  // per byte, with a bias of 0x80 so that no subtraction borrows into the next byte:
  // (i | 0x80) - a keeps bit 7 iff i >= a, and (b | 0x80) - (i + 1) keeps it iff i < b
  const uint32_t A = a * 0x01010101u, B = (b * 0x01010101u) | HI;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t idx = 0x03020100u + 0x04040404u * k;
    const uint32_t in = ((idx | HI) - A) & (B - (idx + 0x01010101u)) & HI;
    m[k] = (in >> 7) * 0xFFu;
  }
}

// Byte masks (0xFF per byte) of the chunk's grid positions in [lo, hi).
__device__ __forceinline__ void range_masks(uint64_t q0, uint64_t lo, uint64_t hi, uint32_t m[4]) {
  const int64_t a64 = (int64_t)lo - (int64_t)q0, b64 = (int64_t)hi - (int64_t)q0;
  const uint32_t a = a64 <= 0 ? 0u : (a64 >= 16 ? 16u : (uint32_t)a64);
  const uint32_t b = b64 <= 0 ? 0u : (b64 >= 16 ? 16u : (uint32_t)b64);
  byte_masks_ab(a, b, m);
}

// range_masks in 32-bit arithmetic, for positions below 2^31 (one wave walking one
// string).
__device__ __forceinline__ void range_masks32(uint32_t q0, uint32_t lo, uint32_t hi, uint32_t m[4]) {
  const int32_t a32 = (int32_t)lo - (int32_t)q0, b32 = (int32_t)hi - (int32_t)q0;
  const uint32_t a = a32 <= 0 ? 0u : (a32 >= 16 ? 16u : (uint32_t)a32);
  const uint32_t b = b32 <= 0 ? 0u : (b32 >= 16 ? 16u : (uint32_t)b32);
  byte_masks_ab(a, b, m);
}

// ================================================================ UTF-8 classification

// Byte classes of Table 1, looked up by the top three bits of each byte with one
// v_perm (an 8-entry byte table).  Flag bits of a class byte:
//   bit 7  ASCII (00..7F)              bit 3  continuation (80..BF)
//   bit 6  2-byte lead (C0..DF)        bit 2  any lead >= C0
//   bit 5  lead >= E0 (3/4-byte)       bit 4  lead >= F0, added by add_f0
// The bit positions are chosen so that "class of the byte d positions back" lands on
// bit 7 after a byte shift by d and a bit shift by d (or by 5 for bit 2).
constexpr uint32_t LUT8_LO = 0x80808080u;  // top bits 000..011: ASCII
constexpr uint32_t LUT8_HI = 0x24440808u;  // 100, 101: continuation; 110: 2-byte lead; 111: >= E0

__device__ __forceinline__ uint32_t cls_lut(uint32_t v) { return perm(LUT8_HI, LUT8_LO, (v >> 5) & 0x07070707u); }
// bit 4 for bytes >= F0: a >= E0 byte whose own bit 4 is set
__device__ __forceinline__ uint32_t f0_bits(uint32_t C, uint32_t v) { return (C >> 1) & v & 0x10101010u; }

// One thread's 16-byte chunk with the 4 bytes before it, and their classes.
struct Chunk8 {
  uint32_t x[4];
  uint32_t xp;
  uint32_t C[4];
  uint32_t Cp;
};

// Wave-uniform content class: 0 = ASCII only, 1 = no byte >= E0, 2 = no byte >= F0,
// 3 = general.  Lower classes skip work that cannot matter for the wave's bytes.
// For class 3 the >= F0 bits are merged into the class bytes.
__device__ __forceinline__ int classify8(Chunk8& c) {
  c.Cp = cls_lut(c.xp);
#pragma unroll
  for (int k = 0; k < 4; ++k) c.C[k] = cls_lut(c.x[k]);
  const uint32_t orc = c.Cp | c.C[0] | c.C[1] | c.C[2] | c.C[3];
  if (!__any((orc & 0x0C0C0C0Cu) != 0)) return 0;
  if (!__any((orc & 0x20202020u) != 0)) return 1;
  // some lead >= E0: look for leads >= F0 (only then are their bits needed)
  const uint32_t fp = f0_bits(c.Cp, c.xp), f0 = f0_bits(c.C[0], c.x[0]), f1 = f0_bits(c.C[1], c.x[1]),
                 f2 = f0_bits(c.C[2], c.x[2]), f3 = f0_bits(c.C[3], c.x[3]);
  if (!__any((fp | f0 | f1 | f2 | f3) != 0)) return 2;
  c.Cp |= fp;
  c.C[0] |= f0;
  c.C[1] |= f1;
  c.C[2] |= f2;
  c.C[3] |= f3;
  return 3;
}

// Per-chunk analysis, and (DECODE) the UTF-16 words of the chunk.
//
// E: bit-7 flag per position that emits one UTF-16 word.  A character emits at its
// last byte, and a 4-byte character also at its third byte (the high surrogate):
// the end mask of section 6.1 in its exact form, where a lead of length L marks the
// position L-1 after it, so E = ascii | lead2 shifted 1 | lead>=E0 shifted 2 |
// lead>=F0 shifted 3.  It depends only on the bytes at or before the position, so
// each character of a valid prefix is counted exactly where its words belong.
//
// det: some position in [0, n] shows that a rule is broken nearby:
//   * continuation bytes must be exactly where the leads' lengths put them: the
//     mismatched-continuation check of section 6.4 (expected: >=C0 one back, >=E0
//     two back, >=F0 three back; compared with "is a continuation");
//   * C0/C1 leads (overlong 2-byte forms, section 6.4);
//   * the second-byte ranges that make 3/4-byte forms overlong, surrogates or larger
//     than U+10FFFF (the range check of section 6.4), on the lead and the next byte.
// Every invalid byte j makes some position in [j, j+3] detect, and every detection
// at p has an invalid byte in [p-3, p]; the exact first error is then found by a
// scalar check of the chunk (locate8).
//
// W[2k], W[2k+1]: the words of positions (4k, 4k+1) and (4k+2, 4k+3) as 16-bit lane
// pairs.  Each position gathers its last, second-last and third-last bytes with the
// tag bits stripped (section 6.2) and sums them as s + 64*s1 + 4096*s2 (mod 2^16);
// s1 counts only at continuation positions and s2 only after a 3/4-byte lead.  The
// sum is assembled bytewise: low byte s | s1<<6, high byte s1>>2 | s2<<4.  The third
// byte of a 4-byte character becomes (sum >> 4) + 0xD7C0 and the fourth sum | 0xDC00
// (the surrogate fix-up of section 6.2, where 0xD7C0 = 0xD800 - 0x40).
template <int CLS, bool DECODE, bool FULL>
__device__ __forceinline__ void process8(const Chunk8& c, const uint32_t inE[4], const uint32_t inD[4],
                                         uint32_t E[4], uint32_t& count, uint32_t& det, uint32_t W[8]) {
  count = 0;
  det = 0;
  uint32_t sp = 0;
  if (DECODE && CLS != 0) sp = c.xp & ~(bytemask(c.xp) & 0xC0C0C0C0u);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t v = c.x[k];
    const uint32_t vp = (k == 0) ? c.xp : c.x[k - 1];
    const uint32_t Ck = c.C[k];
    const uint32_t Cq = (k == 0) ? c.Cp : c.C[k - 1];
    uint32_t e;
    if (CLS == 0) {
      e = HI;
      if (DECODE) {
        W[2 * k] = zx_lo(v);
        W[2 * k + 1] = zx_hi(v);
      }
    } else {
      const uint32_t S1 = abyte(Ck, Cq, 3);
      uint32_t S2 = 0, S3 = 0, u = 0;
      if (CLS >= 2) {
        S2 = abyte(Ck, Cq, 2);
        u = S2 << 2;
        if (CLS == 3) {
          S3 = abyte(Ck, Cq, 1);
          u |= S3 << 3;
        }
      }
      e = (Ck | (S1 << 1) | u) & HI;
      const uint32_t cov = (S1 << 5) | u;
      uint32_t d = ((Ck << 4) ^ cov) & HI;
      // C0/C1: a 2-byte lead whose payload bits 4..1 are zero (zero test lands on bit 6,
      // the 2-byte-lead flag)
      d |= ~((v & 0x1E1E1E1Eu) + 0x3F3F3F3Fu) & Ck & 0x40404040u;
      if (CLS >= 2) {
        // second byte after a 3-byte lead E0..EF: the bad pairs are E0 80..9F and ED A0..BF,
        // i.e. lead nibble 0 when the next byte's bit 5 is clear and 0xD when it is set:
        // (lead ^ (bit5 ? 0xD : 0)) & 0xF == 0.  The zero test lands on bit 5, the
        // lead>=E0 flag of the byte one back.
        const uint32_t y1 = abyte(v, vp, 3);
        const uint32_t k13 = perm(0u, 0x00000D00u, (v >> 5) & 0x01010101u);
        const uint32_t u = (y1 ^ k13) & 0x0F0F0F0Fu;
        uint32_t lead3 = S1;
        if (CLS == 3) lead3 &= ~(S1 << 1);  // exclude >= F0 leads
        d |= ~(u + 0x1F1F1F1Fu) & lead3 & 0x20202020u;
        if (CLS == 3) {
          // after a 4-byte lead F0..FF: with c = bits 5..4 of the next byte, v4 = 4a + c
          // (a = lead & 0xF) is bad exactly when v4 == 0 (F0 80..8F) or v4 >= 17
          // (F4 90.., F5..FF)
          const uint32_t a = y1 & 0x0F0F0F0Fu;
          const uint32_t cc = (v >> 4) & 0x03030303u;
          const uint32_t v4 = (a << 2) + cc;
          d |= ((v4 + 0x6F6F6F6Fu) | ~(v4 + 0x7F7F7F7Fu)) & (S1 << 3) & HI;
        }
      }
      det |= FULL ? d : (d & inD[k]);
      if (DECODE) {
        const uint32_t M1 = bytemask(v);                   // non-ASCII positions
        const uint32_t s = v & ~(M1 & 0xC0C0C0C0u);        // tag bits stripped
        const uint32_t s1 = abyte(s, sp, 3) & M1;          // second-last byte
        const uint32_t lo = s | ((s1 & 0x03030303u) << 6);
        uint32_t hi;
        if (CLS >= 2) {
          // third-last byte after a 3/4-byte lead; only its low nibble survives
          const uint32_t s2 = abyte(v, vp, 2) & bytemask(S2 << 2);
          hi = ((s1 >> 2) & 0x0F0F0F0Fu) | ((s2 << 4) & 0xF0F0F0F0u);
        } else {
          hi = (s1 >> 2) & 0x0F0F0F0Fu;
        }
        uint32_t wl = perm(hi, lo, 0x05010400u);
        uint32_t wh = perm(hi, lo, 0x07030602u);
        if (CLS == 3) {
          const uint32_t fh = S2 << 3;  // >= F0 two back: the high surrogate
          const uint32_t fl = S3 << 3;  // >= F0 three back: the low surrogate
          const us2 hl = (as_us2(wl) >> (us2)(4)) + (us2)(0xD7C0);
          const us2 hh = (as_us2(wh) >> (us2)(4)) + (us2)(0xD7C0);
          const uint32_t mhl = lanemask_lo(fh), mhh = lanemask_hi(fh);
          wl = (as_u32(hl) & mhl) | (wl & ~mhl);
          wh = (as_u32(hh) & mhh) | (wh & ~mhh);
          wl |= lanemask_lo(fl) & 0xDC00DC00u;
          wh |= lanemask_hi(fl) & 0xDC00DC00u;
        }
        W[2 * k] = wl;
        W[2 * k + 1] = wh;
        sp = s;
      }
    }
    if (!FULL) e &= inE[k];
    E[k] = e;
    count += __builtin_popcount(e);
  }
}

// Dispatch on the wave's content class and on whether the chunk lies wholly inside
// the input (then no range masks are applied at all).
template <bool DECODE>
__device__ __forceinline__ void process8_any(int cls, bool full, const Chunk8& c, const uint32_t inE[4],
                                             const uint32_t inD[4], uint32_t E[4], uint32_t& cnt, uint32_t& det,
                                             uint32_t W[8]) {
  if (full) {
    switch (cls) {
      case 0: process8<0, DECODE, true>(c, inE, inD, E, cnt, det, W); break;
      case 1: process8<1, DECODE, true>(c, inE, inD, E, cnt, det, W); break;
      case 2: process8<2, DECODE, true>(c, inE, inD, E, cnt, det, W); break;
      default: process8<3, DECODE, true>(c, inE, inD, E, cnt, det, W); break;
    }
  } else {
    switch (cls) {
      case 0: process8<0, DECODE, false>(c, inE, inD, E, cnt, det, W); break;
      case 1: process8<1, DECODE, false>(c, inE, inD, E, cnt, det, W); break;
      case 2: process8<2, DECODE, false>(c, inE, inD, E, cnt, det, W); break;
      default: process8<3, DECODE, false>(c, inE, inD, E, cnt, det, W); break;
    }
  }
}

// Output words per byte (the length-query formula): one per non-continuation byte
// and one more per byte >= F0.  Counts only positions whose mask byte is set.
__device__ __forceinline__ uint32_t len8_count(const uint32_t x[4], bool full, const uint32_t m[4]) {
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t v = x[k];
    const uint32_t nc = (~v | (v << 1)) & HI;  // not a continuation byte
    const uint32_t f0 = v & (v << 1) & (v << 2) & (v << 3) & HI;
    if (full) cnt += __builtin_popcount(nc) + __builtin_popcount(f0);
    else cnt += __builtin_popcount(nc & m[k]) + __builtin_popcount(f0 & m[k]);
  }
  return cnt;
}

// ================================================================ UTF-8 error location

// Kind of the first rule broken by the character starting at in[i] (i < n): the
// order of the checks follows the scalar decoder (byte type, continuation bytes,
// shortest form / surrogate / U+10FFFF via the second-byte ranges).
__device__ int32_t utf8_kind_at(const uint8_t* in, uint64_t n, uint64_t i) {
  const uint32_t b0 = in[i];
  if (b0 < 0x80) return ST_OK;
  if (b0 < 0xC0) return ST_STRAY_CONT;
  if (b0 < 0xC2) return ST_OVERLONG;
  if (b0 >= 0xF5) return ST_BAD_BYTE;
  const int k = b0 >= 0xF0 ? 3 : (b0 >= 0xE0 ? 2 : 1);
  for (int d = 1; d <= k; ++d) {
    if (i + d >= n || (in[i + d] & 0xC0) != 0x80) return ST_MISSING_CONT;
  }
  const uint32_t b1 = in[i + 1];
  if (b0 == 0xE0 && b1 < 0xA0) return ST_OVERLONG;
  if (b0 == 0xF0 && b1 < 0x90) return ST_OVERLONG;
  if (b0 == 0xED && b1 >= 0xA0) return ST_SURROGATE;
  if (b0 == 0xF4 && b1 >= 0x90) return ST_TOO_LARGE;
  return ST_OK;
}

// Is byte j (< n) the first byte of an invalid character or a stray continuation?
__device__ bool utf8_flag_at(const uint8_t* in, uint64_t n, uint64_t j) {
  const uint32_t b = in[j];
  if ((b & 0xC0) == 0x80) {
    bool cov = (j >= 1 && in[j - 1] >= 0xC0) || (j >= 2 && in[j - 2] >= 0xE0) ||
               (j >= 3 && in[j - 3] >= 0xF0);
    return !cov;
  }
  return utf8_kind_at(in, n, j) != ST_OK;
}

// Exact first invalid byte among logical positions [p_lo, p_hi) clipped to [0, n),
// or NO_ERR.  Used only for chunks whose analysis detected something.
__device__ uint64_t locate8(const uint8_t* in, uint64_t n, int64_t p_lo, int64_t p_hi) {
  if (p_lo < 0) p_lo = 0;
  if (p_hi > (int64_t)n) p_hi = (int64_t)n;
  for (int64_t j = p_lo; j < p_hi; ++j) {
    if (utf8_flag_at(in, n, (uint64_t)j)) return (uint64_t)j;
  }
  return NO_ERR;
}

// ================================================================ UTF-16 side

// 8 words at grid position q0 (in words, a multiple of 8).  Words outside the input
// read as 0.
__device__ __forceinline__ void load16(const Launch& L, uint64_t q0, uint32_t x[4]) {
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const uint16_t* b = reinterpret_cast<const uint16_t*>(L.base);
  if (q0 >= lo && q0 + 8 <= hi) {
    uint4 v = *reinterpret_cast<const uint4*>(b + q0);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else {
    x[0] = x[1] = x[2] = x[3] = 0;
    if (q0 + 8 <= lo || q0 >= hi) return;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      uint64_t q = q0 + i;
      if (q >= lo && q < hi) x[i >> 1] |= (uint32_t)b[q] << (16 * (i & 1));
    }
  }
  if (L.be) {
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = bswap16x2(x[k]);
  }
}

__device__ __forceinline__ uint32_t load16_prev(const Launch& L, uint64_t q0) {
  if (q0 == 0) return 0;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const uint64_t q = q0 - 1;
  const uint16_t* b = reinterpret_cast<const uint16_t*>(L.base);
  if (!(q >= lo && q < hi)) return 0u;
  return L.be ? bswap16(b[q]) : (uint32_t)b[q];
}

__device__ __forceinline__ bool is_hi(uint32_t w) { return (w & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_lo(uint32_t w) { return (w & 0xFC00u) == 0xDC00u; }

// UTF-8 bytes per UTF-16 word (section 7.3: 1, 2 or 3 bytes; each half of a surrogate
// pair accounts for 2 of the pair's 4 bytes).
__device__ __forceinline__ uint32_t len16(uint32_t w) {
  return w < 0x80u ? 1u : ((w < 0x800u || (w & 0xF800u) == 0xD800u) ? 2u : 3u);
}

// UTF-8 bytes of one word, little-endian in a dword (Figure 1(a)).  The 3-byte form
// [E0|w>>12, 80|(w>>6 & 3F), 80|(w & 3F)] is built once; the 2-byte form is its last
// two bytes with the lead tag raised from 80 to C0, and ASCII is the word itself.  A
// high surrogate emits the first two bytes of its character, which depend on it alone:
// with u = (hi & 0x3FF) + 0x40 = code point >> 10 they are F0|u>>8 and 80|(u>>2 & 3F).
// A low surrogate emits the last two, using the two low bits of the high one.
template <bool SURR>
__device__ __forceinline__ uint32_t enc16(uint32_t w, uint32_t prev, uint32_t c) {
  const uint32_t t3 = 0x008080E0u | (w >> 12) | ((w << 2) & 0x3F00u) | ((w << 16) & 0x3F0000u);
  uint32_t r = (c == 3) ? t3 : ((c == 2) ? ((t3 >> 8) | 0x40u) : w);
  if (SURR) {
    const uint32_t u = (w & 0x3FFu) + 0x40u;
    const uint32_t th = (0xF0u | (u >> 8)) | ((0x80u | ((u >> 2) & 0x3Fu)) << 8);
    const uint32_t tl = 0x8080u | ((prev & 3u) << 4) | ((w >> 6) & 0xFu) | ((w & 0x3Fu) << 8);
    r = is_hi(w) ? th : r;
    r = is_lo(w) ? tl : r;
  }
  return r;
}

// Two words at a time (16-bit lanes of a dword), for chunks wholly inside the input
// in waves without surrogates.  Output bytes per word: 1 + [w >= 0x80] + [w >= 0x800].
__device__ __forceinline__ uint32_t pk_len16(uint32_t X) {
  const us2 w = as_us2(X);
  return pk_nz(as_u32(w >> (us2)(7))) + pk_nz(as_u32(w >> (us2)(11))) + 0x00010001u;
}

// UTF-8 bytes of the two words of X (little-endian in a dword each), given their
// lengths c (1..3).  The 3-byte form [E0|w>>12, 80|(w>>6 & 3F), 80|(w & 3F)] is built
// lane-wise and spread to bytes with v_perm; the 2-byte form is its last two bytes
// with the lead tag raised to C0; ASCII is the word itself.
__device__ __forceinline__ void pk_enc16(uint32_t X, uint32_t c_lo, uint32_t c_hi, uint32_t& v_lo, uint32_t& v_hi) {
  const us2 w = as_us2(X);
  const uint32_t p0 = as_u32(w >> (us2)(12)) | 0x00E000E0u;
  const uint32_t p1 = (as_u32(w >> (us2)(6)) & 0x003F003Fu) | 0x00800080u;
  const uint32_t p2 = (X & 0x003F003Fu) | 0x00800080u;
  const uint32_t q12 = p1 | (p2 << 8);          // bytes: p1.lo, p2.lo, p1.hi, p2.hi
  const uint32_t q12c = q12 | 0x00400040u;      // p1 with the 2-byte lead tag C0
  const uint32_t t3l = perm(q12, p0, 0x0C050400u), t3h = perm(q12, p0, 0x0C070602u);
  const uint32_t t2l = perm(q12c, 0u, 0x0C0C0504u), t2h = perm(q12c, 0u, 0x0C0C0706u);
  v_lo = c_lo == 3 ? t3l : (c_lo == 2 ? t2l : (X & 0xFFFFu));
  v_hi = c_hi == 3 ? t3h : (c_hi == 2 ? t2h : (X >> 16));
}

// Does any of the chunk's words (or the word before it) lie in U+D800..DFFF?
__device__ __forceinline__ bool any_surrogate(const uint32_t x[4], uint32_t wp) {
  uint32_t m = ((wp & 0xF800u) == 0xD800u) ? 1u : 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t z = (x[k] ^ 0xD800D800u) & 0xF800F800u;
    m |= ((z & 0xFFFFu) == 0u || (z >> 16) == 0u) ? 1u : 0u;
  }
  return m != 0;
}

// Exact first unpaired surrogate among [p_lo, p_hi) clipped to [0, n) (sections 2.1, 7.4).
__device__ uint64_t locate16(const uint16_t* in, uint64_t n, int64_t p_lo, int64_t p_hi, bool be = false) {
  if (p_lo < 0) p_lo = 0;
  if (p_hi > (int64_t)n) p_hi = (int64_t)n;
  auto rd = [&](int64_t j) { return be ? bswap16(in[j]) : (uint32_t)in[j]; };
  for (int64_t j = p_lo; j < p_hi; ++j) {
    const uint32_t w = rd(j);
    if (is_hi(w) && ((uint64_t)j + 1 >= n || !is_lo(rd(j + 1)))) return (uint64_t)j;
    if (is_lo(w) && (j == 0 || !is_hi(rd(j - 1)))) return (uint64_t)j;
  }
  return NO_ERR;
}

// Per chunk of 8 words: output bytes per word (0 outside the input) and detection of
// unpaired surrogates: position p detects when "p is a low surrogate" differs from
// "p-1 is a high surrogate" (the sequencing check of section 7.4, with the carry of
// the previous chunk taken from the neighbouring word).  Returns whether any word of
// the chunk or its predecessor is a surrogate.
template <bool FULL>
__device__ __forceinline__ bool analyze16(const uint32_t x[4], uint32_t wp, uint64_t q0, uint64_t lo, uint64_t hi,
                                          uint32_t len[8], uint32_t& cnt, bool& det) {
  cnt = 0;
  uint32_t d = 0, sur = (wp & 0xF800u) == 0xD800u ? 1u : 0u;
  uint32_t prev = wp;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t w = (x[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
    const uint32_t s = (w & 0xF800u) == 0xD800u ? 1u : 0u;
    uint32_t c = 1u + (w >= 0x80u ? 1u : 0u) + (w >= 0x800u ? 1u : 0u) - s;
    uint32_t dd = (is_lo(w) != is_hi(prev)) ? 1u : 0u;
    if (!FULL) {
      const uint64_t q = q0 + j;
      c = (q >= lo && q < hi) ? c : 0u;
      dd = (q >= lo && q <= hi) ? dd : 0u;
    }
    len[j] = c;
    cnt += c;
    d |= dd;
    sur |= s;
    prev = w;
  }
  det = d != 0;
  return sur != 0;
}

// ================================================================ shared plumbing

// Segment i is workgroup i.  Workgroups are dispatched in increasing order on each
// XCD, so every predecessor a look-back waits for has been dispatched or will be once
// smaller workgroups on its XCD finish; each of those waits only on smaller segments,
// so every wait ends.  (The look-back watchdog bounds each wait regardless.)  No fences
// and no single-address counters in the per-segment path: cross-segment data goes
// through self-contained 64-bit status words, and the result is assembled by a
// separate one-workgroup finalisation kernel after the launch boundary.

__device__ __forceinline__ uint32_t ld_fault(WsHeader* ws) {
  return __hip_atomic_load(&ws->fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Finalisation epilogue (one thread): make the workspace ready for the next launch.
// The fault flag is cleared too: a watchdog trip is reported by the launch it happened
// in, and the next launch carries a new epoch, so no status word of the failed launch
// is ever read again.
__device__ __forceinline__ void reset_ws(WsHeader* ws) {
  st_agent(&ws->err, NO_ERR);
  st_agent(&ws->acc, 0);
  __hip_atomic_store(&ws->fault, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t ep = __hip_atomic_load(&ws->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&ws->epoch, (ep + 1) & EPOCH_MASK, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void write_result(void* r, int32_t st, uint64_t count, uint64_t written) {
  Result* res = reinterpret_cast<Result*>(r);
  res->status = st;
  res->reserved = 0;
  res->count = count;
  res->written = written;
}

__device__ __forceinline__ uint32_t cur_epoch(WsHeader* ws) {
  return __hip_atomic_load(&ws->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads chunk q0 of a UTF-8 input with its halo and range masks.
template <int WG>
__device__ __forceinline__ bool chunk8(const Launch& L, uint64_t q0, const uint32_t x[4], Chunk8& c,
                                       uint32_t inE[4], uint32_t inD[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) c.x[k] = x[k];
  c.xp = __shfl_up(x[3], 1, 64);
  if ((threadIdx.x & 63) == 0) c.xp = load8_prev(L, q0);
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const bool full = q0 >= lo && q0 + 16 <= hi;
  if (!full) {
    range_masks(q0, lo, hi, inE);
    range_masks(q0, lo, hi + 1, inD);
  }
  return full;
}

// ================================================================ length queries

// Section 6.2 / 7.3 output-length formula, summed; no validation.  Each segment
// stores its partial sum in its status word; k_fin_len adds them up.
template <int WG>
__global__ void __launch_bounds__(WG) k_len8(Launch L) {
  constexpr uint64_t T = 16ull * WG;
  __shared__ unsigned long long lds[WG / 64 + 2];
  const uint64_t seg = blockIdx.x;
  const uint64_t q00 = seg * L.seg * T + 16ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  uint32_t x[4], xn[4], m[4];
  load8(L, q00, x);
  uint32_t acc = 0;
  for (uint32_t s = 0; s < L.seg; ++s) {
    const uint64_t q0 = q00 + s * T;
    if (s + 1 < L.seg) load8(L, q0 + T, xn);
    const bool full = q0 >= lo && q0 + 16 <= hi;
    if (!full) range_masks(q0, lo, hi, m);
    acc += len8_count(x, full, m);
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = xn[k];
  }
  const uint64_t sum = block_sum_u64<WG>(acc, lds);
  if (threadIdx.x == 0) L.status[seg] = sum;
}

template <int WG>
__global__ void __launch_bounds__(WG) k_len16(Launch L) {
  constexpr uint64_t TW = 8ull * WG;
  __shared__ unsigned long long lds[WG / 64 + 2];
  const uint64_t seg = blockIdx.x;
  const uint64_t q00 = seg * L.seg * TW + 8ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  uint32_t x[4], xn[4];
  load16(L, q00, x);
  uint32_t acc = 0;
  for (uint32_t s = 0; s < L.seg; ++s) {
    const uint64_t q0 = q00 + s * TW;
    if (s + 1 < L.seg) load16(L, q0 + TW, xn);
    const bool full = q0 >= lo && q0 + 8 <= hi;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t w = (x[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
      acc += (full || (q0 + j >= lo && q0 + j < hi)) ? len16(w) : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = xn[k];
  }
  const uint64_t sum = block_sum_u64<WG>(acc, lds);
  if (threadIdx.x == 0) L.status[seg] = sum;
}

template <int WG>
__global__ void __launch_bounds__(WG) k_fin_len(Launch L) {
  __shared__ unsigned long long lds[WG / 64 + 2];
  uint64_t s = 0;
  for (uint64_t t = threadIdx.x; t < L.ntiles; t += WG) s += L.status[t];
  s = block_sum_u64<WG>(s, lds);
  if (threadIdx.x == 0) {
    write_result(L.result, ld_fault(L.ws) ? ST_DEVICE : ST_OK, s, s);
    reset_ws(L.ws);
  }
}

// ================================================================ validation

template <int WG>
__global__ void __launch_bounds__(WG) k_validate8(Launch L) {
  constexpr uint64_t T = 16ull * WG;
  __shared__ unsigned long long werr;  // the workgroup's first error (see report_err)
  const uint64_t seg = blockIdx.x;
  const uint64_t q00 = seg * L.seg * T + 16ull * threadIdx.x;
  uint32_t x[4], xn[4], inE[4], inD[4], E[4], W[8], cnt, det;
  Chunk8 c;
  if (threadIdx.x == 0) werr = NO_ERR;
  load8(L, q00, x);
  __syncthreads();
  for (uint32_t s = 0; s < L.seg; ++s) {
    const uint64_t q0 = q00 + s * T;
    if (s + 1 < L.seg) load8(L, q0 + T, xn);
    const bool full = chunk8<WG>(L, q0, x, c, inE, inD);
    const int cls = classify8(c);
    process8_any<false>(cls, full, c, inE, inD, E, cnt, det, W);
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)L.mis;
      if (before(p0 - 3, werr)) {
        const uint64_t e = locate8(L.base + L.mis, L.n, p0 - 3, p0 + 16);
        if (e != NO_ERR) atomicMin(&werr, (unsigned long long)e);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = xn[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) report_err(L.err, werr);
}

__global__ void k_fin_validate8(Launch L) {
  if (threadIdx.x == 0) {
    const uint64_t err = ld_agent(L.err);
    if (ld_fault(L.ws)) write_result(L.result, ST_DEVICE, 0, 0);
    else if (err != NO_ERR) write_result(L.result, utf8_kind_at(L.base + L.mis, L.n, err), err, err);
    else write_result(L.result, ST_OK, L.n, L.n);
    reset_ws(L.ws);
  }
}

template <int WG>
__global__ void __launch_bounds__(WG) k_validate16(Launch L) {
  constexpr uint64_t TW = 8ull * WG;
  __shared__ unsigned long long werr;  // the workgroup's first error (see report_err)
  const uint64_t seg = blockIdx.x;
  const uint64_t q00 = seg * L.seg * TW + 8ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  uint32_t x[4], xn[4], len[8], cnt;
  bool det;
  if (threadIdx.x == 0) werr = NO_ERR;
  load16(L, q00, x);
  __syncthreads();
  for (uint32_t s = 0; s < L.seg; ++s) {
    const uint64_t q0 = q00 + s * TW;
    if (s + 1 < L.seg) load16(L, q0 + TW, xn);
    uint32_t wp = __shfl_up(x[3] >> 16, 1, 64);
    if ((threadIdx.x & 63) == 0) wp = load16_prev(L, q0);
    if (q0 >= lo && q0 + 8 <= hi) analyze16<true>(x, wp, q0, lo, hi, len, cnt, det);
    else analyze16<false>(x, wp, q0, lo, hi, len, cnt, det);
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)L.mis;
      if (before(p0 - 1, werr)) {
        const uint16_t* in = reinterpret_cast<const uint16_t*>(L.base) + L.mis;
        const uint64_t e = locate16(in, L.n, p0 - 1, p0 + 8, L.be != 0);
        if (e != NO_ERR) atomicMin(&werr, (unsigned long long)e);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = xn[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) report_err(L.err, werr);
}

__global__ void k_fin_validate16(Launch L) {
  if (threadIdx.x == 0) {
    const uint64_t err = ld_agent(L.err);
    if (ld_fault(L.ws)) write_result(L.result, ST_DEVICE, 0, 0);
    else if (err != NO_ERR) write_result(L.result, ST_SURROGATE, err, err);
    else write_result(L.result, ST_OK, L.n, L.n);
    reset_ws(L.ws);
  }
}

// Workspace initialisation (called once per context, outside any capture).
__global__ void k_ws_init(WsHeader* ws) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ws->spare0 = 0;
    ws->spare1 = 0;
    ws->err = NO_ERR;
    ws->acc = 0;
    ws->epoch = 1;
    ws->fault = 0;
  }
}

}  // namespace utfx_dev
