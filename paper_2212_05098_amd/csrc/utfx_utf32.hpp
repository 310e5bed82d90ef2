// UTF-32LE: one 32-bit unit per character (section 2).  The kernels reuse the
// single-buffer machinery of UTF-16: segments of S tiles per workgroup, one read, a scan
// of per-chunk output counts, the decoupled look-back, output staged in LDS and stored
// with coalesced 16-byte stores, the UTF-8 classification and validation of section 6.4
// (classify8 / process8 / locate8), and the same result convention.
//
//   UTF-8 -> UTF-32: a character's code point is emitted at its last byte, from the
//   payload bits of its 1-4 bytes (Figure 1(a)); a chunk's count is its number of
//   non-continuation bytes, so characters that start in the 3 bytes before a chunk and
//   end inside it are emitted by that chunk (spill8_chars).
//   UTF-32 -> UTF-8 / UTF-16: each unit is a character by itself; a unit in U+D800..DFFF
//   or above U+10FFFF is an error at its own offset (section 2), and the others are
//   encoded by Figure 1(a) or as one word / a surrogate pair (section 2.1).
//   UTF-16 -> UTF-32: a pair is emitted once, at its low surrogate; pairing is checked
//   as in UTF-16 -> UTF-8 (section 7.4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "utfx_device.hpp"
#include "utfx_kernels.hpp"
#include "utfx_transcode.hpp"

namespace utfx_dev {

// ================================================================ UTF-8 -> UTF-32LE

// Characters starting in a 16-byte chunk: its bytes that are not continuation bytes
// (positions whose mask byte is clear count 0).
__device__ __forceinline__ uint32_t count8_chars(const uint32_t x[4], const uint32_t* m) {
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t nc = (~x[k] | (x[k] << 1)) & HI;  // bit 7: not 10xxxxxx
    if (m) nc &= m[k];
    acc += __builtin_popcount(nc);
  }
  return acc;
}

// Characters that start in the 3 bytes before a chunk and end inside it: a lead one
// back, a lead >= E0 two back, a lead >= F0 three back (xp: the 4 bytes before).
__device__ __forceinline__ uint32_t spill8_chars(uint32_t xp) {
  return ((xp >> 24) >= 0xC0u) + (((xp >> 16) & 0xFFu) >= 0xE0u) + (((xp >> 8) & 0xFFu) >= 0xF0u);
}

// One 16-byte chunk: validate and decode it with process8 (the UTF-16 words of section
// 6.2 at each emit position), then scatter the code point of every character that ends
// in it into the stage from slot PAD + off - spill on.  A BMP character's word is its
// code point; a 4-byte character is emitted once, at its low surrogate, as 0x10000 +
// (high - 0xD800) * 1024 + (low - 0xDC00), the high surrogate being the word one
// position back (for position 0, in the previous chunk, its code point comes straight
// from the four bytes, Figure 1(a)).  Returns the slot after the chunk's last code point
// (LIM for a chunk whose slots would leave the stage, which then writes to the dump slot).
template <uint32_t PAD, uint32_t LIM, uint32_t DUMP>
__device__ __forceinline__ uint32_t chunk_u8_to_u32(const uint32_t x[4], uint32_t xp, bool full, uint64_t q0,
                                                    uint64_t lo, uint64_t hi, uint32_t off, uint32_t* stage,
                                                    uint32_t* first, uint32_t* det_out) {
  Chunk8 ch;
#pragma unroll
  for (int i = 0; i < 4; ++i) ch.x[i] = x[i];
  ch.xp = xp;
  uint32_t inE[4], inD[4], E[4], W[8], cnt, det;
  if (!full) {
    range_masks(q0, lo, hi, inE);
    range_masks(q0, lo, hi + 1, inD);
  }
  const int cls = classify8(ch);
  process8_any<true>(cls, full, ch, inE, inD, E, cnt, det, W);
  const uint32_t idx = PAD + off - spill8_chars(xp);
  *first = idx;
  const bool fits = idx + 16 <= LIM;
  uint32_t* pw = stage + (fits ? idx : DUMP);
  uint32_t* const dump = stage + DUMP;
  // position 0 as the end of a 4-byte character whose first three bytes are in xp
  const uint32_t cp0 = ((xp >> 8) & 0x07u) << 18 | ((xp >> 16) & 0x3Fu) << 12 | ((xp >> 24) & 0x3Fu) << 6 |
                       (x[0] & 0x3Fu);
  uint32_t prev = 0;  // the word one position back
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const uint32_t pair = W[p >> 1];
    const uint32_t w = (p & 1) ? (pair >> 16) : (pair & 0xFFFFu);
    const uint32_t e = (E[p >> 2] >> (8 * (p & 3) + 7)) & 1u;
    const bool hi_half = (w & 0xFC00u) == 0xD800u, lo_half = (w & 0xFC00u) == 0xDC00u;
    const uint32_t cp4 = (p == 0) ? cp0 : 0x10000u + ((prev - 0xD800u) << 10) + (w - 0xDC00u);
    const uint32_t cp = lo_half ? cp4 : w;
    const uint32_t bit = (e && !hi_half) ? 1u : 0u;
    *(bit ? pw : dump) = cp;
    pw += bit;
    prev = w;
  }
  *det_out = det;
  return fits ? (uint32_t)(pw - stage) : LIM;
}

template <int WG, int S>
struct Seg32Smem {
  static constexpr int NW = WG / 64;
  static constexpr uint32_t SEGB = 16u * WG * S;
  static constexpr uint32_t PAD = 16;
  static constexpr uint32_t LIM = PAD + SEGB;
  static constexpr uint32_t DUMP = LIM + 16;
  static constexpr uint32_t SSZ = DUMP + 20;
  uint32_t stage[SSZ];
  uint32_t wtot[NW * (S / 2)];
  uint32_t halo[S * NW];
  unsigned long long seg_base;
  unsigned long long werr;
  uint32_t bounds[2];
};

template <int WG, int S>
__global__ void __launch_bounds__(WG) k_u8_to_u32(Launch L) {
  typedef Seg32Smem<WG, S> M;
  __shared__ __attribute__((aligned(16))) M sm;
  constexpr int NW = M::NW;
  constexpr uint32_t T = 16u * WG;
  constexpr uint32_t SEGB = M::SEGB;
  constexpr uint32_t PAD = M::PAD, LIM = M::LIM, DUMP = M::DUMP;
  const uint64_t seg = blockIdx.x;
  uint32_t x[S][4];
  load_seg8<WG, S>(L, seg, x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t epoch = cur_epoch(L.ws);
  const uint64_t s0 = seg * SEGB;
  const uint64_t q00 = s0 + 16ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const bool segfull = s0 >= lo && s0 + SEGB <= hi;

  // ---- count, scan, publish
  const uint32_t xp_seg = (threadIdx.x == 0) ? load8_prev(L, s0) : 0u;
  uint32_t c[S];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * T;
    if (segfull || (q0 >= lo && q0 + 16 <= hi)) {
      c[k] = count8_chars(x[k], nullptr);
    } else {
      uint32_t m[4];
      range_masks(q0, lo, hi, m);
      c[k] = count8_chars(x[k], m);
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < S; ++k) sm.halo[k * NW + wid] = x[k][3];
  }
  if (threadIdx.x == 0) sm.werr = NO_ERR;
  uint32_t off[S];
  const uint32_t seg_total = segment_offsets<WG, S>(c, off, sm.wtot);  // contains a barrier
  if (threadIdx.x == 0) {
    debug_delay(L.dbg, seg);
    publish_aggregate(L.status, seg, seg_total, epoch);
  }

  // ---- validate, decode, scatter into the stage
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * T;
    const uint32_t hl = (wid > 0) ? sm.halo[k * NW + wid - 1] : (k > 0 ? sm.halo[(k - 1) * NW + NW - 1] : xp_seg);
    uint32_t first, det;
    const bool full = segfull || (q0 >= lo && q0 + 16 <= hi);
    const uint32_t idx = chunk_u8_to_u32<PAD, LIM, DUMP>(x[k], wave_shr1(x[k][3], hl), full, q0, lo, hi, off[k],
                                                         sm.stage, &first, &det);
    if (k == 0 && threadIdx.x == 0) sm.bounds[0] = first;
    if (k == S - 1 && threadIdx.x == WG - 1) sm.bounds[1] = idx;
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)L.mis;
      if (before(p0 - 3, sm.werr)) {
        const uint64_t e = locate8(L.base + L.mis, L.n, p0 - 3, p0 + 16);
        if (e != NO_ERR) atomicMin(&sm.werr, (unsigned long long)e);
      }
    }
  }
  if (wid == 0) {
    const uint64_t b = lookback_wave(L.status, seg, seg_total, epoch, L.ws, [&](uint64_t j) {
      return wave_segment_sum(j, SEGB, 16, [&](uint64_t q) {
        uint32_t xx[4], mm[4];
        load8(L, q, xx);
        range_masks(q, lo, hi, mm);
        return (uint64_t)count8_chars(xx, mm);
      });
    });
    if (lane == 0) sm.seg_base = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) report_err(L.err, sm.werr);
  const uint32_t st0 = sm.bounds[0];
  uint32_t st1 = sm.bounds[1];
  st1 = st1 < st0 ? st0 : (st1 > LIM ? LIM : st1);
  const int64_t g = (int64_t)sm.seg_base + (int64_t)st0 - (int64_t)PAD;
  store_span<uint32_t>(sm.stage, st0, st1 - st0, reinterpret_cast<uint32_t*>(L.out), (uint64_t)g, L.cap,
                       threadIdx.x, WG);
}

// Result of a UTF-8 -> UTF-32 launch: error kind and the characters of the valid prefix
// (the exclusive prefix of its segment plus the non-continuation bytes of the segment
// before the error), or the total against cap.
template <int WG>
__global__ void __launch_bounds__(WG) k_fin_u8u32(Launch L) {
  __shared__ unsigned long long lds[WG / 64 + 2];
  constexpr uint64_t T = 16ull * WG;
  const uint64_t err = ld_agent(L.err);
  const bool fault = ld_fault(L.ws) != 0;
  uint64_t written = 0;
  if (!fault && err != NO_ERR) {
    const uint64_t qoff = err + L.mis;
    const uint64_t seg = qoff / L.seg_units;
    uint32_t acc = 0;
    uint32_t x[4], m[4];
    for (uint64_t q0b = seg * L.seg_units; q0b < qoff; q0b += T) {
      const uint64_t q0 = q0b + 16ull * threadIdx.x;
      load8(L, q0, x);
      range_masks(q0, L.mis, qoff, m);
      acc += count8_chars(x, m);
    }
    const uint64_t s = block_sum_u64<WG>(acc, lds);
    written = (seg ? tile_inclusive(L.status, seg - 1) : 0) + s;
  }
  __syncthreads();  // every wave has read err and fault before thread 0 resets them
  if (threadIdx.x == 0) {
    const uint64_t tot = tile_inclusive(L.status, L.ntiles - 1);
    if (fault) write_result(L.result, ST_DEVICE, 0, 0);
    else if (err != NO_ERR) write_result(L.result, utf8_kind_at(L.base + L.mis, L.n, err), err, written);
    else if (tot > L.cap) write_result(L.result, ST_OUTPUT_TOO_SMALL, tot, 0);
    else write_result(L.result, ST_OK, tot, tot);
    reset_ws(L.ws);
  }
}

// ================================================================ UTF-32LE side

// 4 units at grid position q0 (in units, a multiple of 4).  Units outside the input
// read as 0.
__device__ __forceinline__ void load32(const Launch& L, uint64_t q0, uint32_t x[4]) {
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const uint32_t* b = reinterpret_cast<const uint32_t*>(L.base);
  if (q0 >= lo && q0 + 4 <= hi) {
    const uint4 v = *reinterpret_cast<const uint4*>(b + q0);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = (q0 + i >= lo && q0 + i < hi) ? b[q0 + i] : 0u;
  }
}

// Section 2: a unit is a character if it is at most U+10FFFF and not a surrogate.
__device__ __forceinline__ bool bad32(uint32_t u) { return (u >= 0xD800u && u <= 0xDFFFu) || u > 0x10FFFFu; }

// UTF-8 bytes of a unit (Figure 1(a)); units above U+FFFF count 4 whether valid or not.
__device__ __forceinline__ uint32_t len32(uint32_t u) {
  return u < 0x80u ? 1u : (u < 0x800u ? 2u : (u < 0x10000u ? 3u : 4u));
}

// UTF-16 words of a unit (section 2.1): two above U+FFFF, whether valid or not.
__device__ __forceinline__ uint32_t len32w(uint32_t u) { return u > 0xFFFFu ? 2u : 1u; }

// Output units (UTF-8 bytes, or UTF-16 words with OUT16) of the in-range units of a
// chunk, and the first invalid in-range unit (4 = none).
template <bool OUT16 = false>
__device__ __forceinline__ uint32_t count32(const uint32_t x[4], uint64_t q0, uint64_t lo, uint64_t hi, bool full,
                                           uint32_t* first_bad) {
  uint32_t acc = 0, fb = 4;
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    const bool in = full || (q0 + i >= lo && q0 + i < hi);
    acc += in ? (OUT16 ? len32w(x[i]) : len32(x[i])) : 0u;
    if (in && bad32(x[i])) fb = (uint32_t)i;
  }
  *first_bad = fb;
  return acc;
}

template <int WG, int S, typename U>
struct Seg32OutSmem {
  static constexpr int NW = WG / 64;
  static constexpr uint32_t PAD = 16;
  static constexpr uint32_t SEGO = (16u / sizeof(U)) * WG * S;  // bound on a segment's output units
  U stage[PAD + SEGO + 32];
  uint32_t wtot[NW * (S / 2)];
  unsigned long long seg_base;
  unsigned long long werr;
};

// UTF-32 -> UTF-8 (U = uint8_t, Figure 1(a)) or UTF-16 (U = uint16_t, section 2.1; the
// words byte-swapped for UTF-16BE when L.be).
template <int WG, int S, typename U>
__global__ void __launch_bounds__(WG) k_u32_to(Launch L) {
  constexpr bool OUT16 = sizeof(U) == 2;
  typedef Seg32OutSmem<WG, S, U> M;
  __shared__ __attribute__((aligned(16))) M sm;
  constexpr uint32_t T = 4u * WG;  // units per tile
  constexpr uint32_t SEGU = T * S;
  constexpr uint32_t PAD = M::PAD;
  const uint64_t seg = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t epoch = cur_epoch(L.ws);
  const uint64_t s0 = seg * SEGU;
  const uint64_t q00 = s0 + 4ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const bool segfull = s0 >= lo && s0 + SEGU <= hi;
  uint32_t x[S][4], c[S], fb[S];
#pragma unroll
  for (int k = 0; k < S; ++k) load32(L, q00 + (uint64_t)k * T, x[k]);
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * T;
    c[k] = count32<OUT16>(x[k], q0, lo, hi, segfull || (q0 >= lo && q0 + 4 <= hi), &fb[k]);
  }
  if (threadIdx.x == 0) sm.werr = NO_ERR;
  uint32_t off[S];
  const uint32_t seg_total = segment_offsets<WG, S>(c, off, sm.wtot);  // contains a barrier
  if (threadIdx.x == 0) {
    debug_delay(L.dbg, seg);
    publish_aggregate(L.status, seg, seg_total, epoch);
  }

  // ---- encode into the stage; the first invalid unit of a chunk is exact
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * T;
    U* p = sm.stage + PAD + off[k];
    const bool full = segfull || (q0 >= lo && q0 + 4 <= hi);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t u = x[k][i];
      const bool in = full || (q0 + i >= lo && q0 + i < hi);
      const uint32_t n = in ? (OUT16 ? len32w(u) : len32(u)) : 0u;
      if (OUT16) {
        if (n == 1) {
          p[0] = (U)u;
        } else if (n == 2) {
          const uint32_t v = u - 0x10000u;
          p[0] = (U)(0xD800u + ((v >> 10) & 0x3FFu));
          p[1] = (U)(0xDC00u + (v & 0x3FFu));
        }
      } else if (n == 1) {
        p[0] = (uint8_t)u;
      } else if (n == 2) {
        p[0] = (uint8_t)(0xC0u | (u >> 6));
        p[1] = (uint8_t)(0x80u | (u & 0x3Fu));
      } else if (n == 3) {
        p[0] = (uint8_t)(0xE0u | (u >> 12));
        p[1] = (uint8_t)(0x80u | ((u >> 6) & 0x3Fu));
        p[2] = (uint8_t)(0x80u | (u & 0x3Fu));
      } else if (n == 4) {
        p[0] = (uint8_t)(0xF0u | ((u >> 18) & 0x07u));
        p[1] = (uint8_t)(0x80u | ((u >> 12) & 0x3Fu));
        p[2] = (uint8_t)(0x80u | ((u >> 6) & 0x3Fu));
        p[3] = (uint8_t)(0x80u | (u & 0x3Fu));
      }
      p += n;
    }
    if (fb[k] < 4) {
      const uint64_t e = q0 + fb[k] - lo;
      if (before((int64_t)e, sm.werr)) atomicMin(&sm.werr, (unsigned long long)e);
    }
  }
  if (wid == 0) {
    const uint64_t b = lookback_wave(L.status, seg, seg_total, epoch, L.ws, [&](uint64_t j) {
      return wave_segment_sum(j, SEGU, 4, [&](uint64_t q) {
        uint32_t xx[4], fbx;
        load32(L, q, xx);
        return (uint64_t)count32<OUT16>(xx, q, lo, hi, false, &fbx);
      });
    });
    if (lane == 0) sm.seg_base = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) report_err(L.err, sm.werr);
  store_span<U>(sm.stage, PAD, seg_total, reinterpret_cast<U*>(L.out), sm.seg_base, L.cap, threadIdx.x, WG,
                L.be != 0);
}

// Result of a UTF-32 -> UTF-8 (UTF-16 with OUT16) launch: the kind of the first invalid
// unit and the output units of the units before it, or the total against cap.
template <int WG, bool OUT16>
__global__ void __launch_bounds__(WG) k_fin_u32to(Launch L) {
  __shared__ unsigned long long lds[WG / 64 + 2];
  constexpr uint64_t T = 4ull * WG;
  const uint64_t err = ld_agent(L.err);
  const bool fault = ld_fault(L.ws) != 0;
  uint64_t written = 0;
  if (!fault && err != NO_ERR) {
    const uint64_t qoff = err + L.mis;
    const uint64_t seg = qoff / L.seg_units;
    uint32_t acc = 0;
    for (uint64_t q0b = seg * L.seg_units; q0b < qoff; q0b += T) {
      const uint64_t q0 = q0b + 4ull * threadIdx.x;
      uint32_t x[4], fb;
      load32(L, q0, x);
      acc += count32<OUT16>(x, q0, L.mis, qoff, false, &fb);
    }
    const uint64_t s = block_sum_u64<WG>(acc, lds);
    written = (seg ? tile_inclusive(L.status, seg - 1) : 0) + s;
  }
  __syncthreads();  // every wave has read err and fault before thread 0 resets them
  if (threadIdx.x == 0) {
    const uint64_t tot = tile_inclusive(L.status, L.ntiles - 1);
    if (fault) {
      write_result(L.result, ST_DEVICE, 0, 0);
    } else if (err != NO_ERR) {
      const uint32_t u = reinterpret_cast<const uint32_t*>(L.base)[L.mis + err];
      write_result(L.result, (u >= 0xD800u && u <= 0xDFFFu) ? ST_SURROGATE : ST_TOO_LARGE, err, written);
    } else if (tot > L.cap) {
      write_result(L.result, ST_OUTPUT_TOO_SMALL, tot, 0);
    } else {
      write_result(L.result, ST_OK, tot, tot);
    }
    reset_ws(L.ws);
  }
}

// ================================================================ UTF-16LE -> UTF-32LE

// Characters starting in an 8-word chunk: its in-range words that are not low
// surrogates.
__device__ __forceinline__ uint32_t count16_chars(const uint32_t x[4], uint64_t q0, uint64_t lo, uint64_t hi,
                                                  bool full) {
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t w = (x[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
    const bool in = full || (q0 + j >= lo && q0 + j < hi);
    acc += (in && !is_lo(w)) ? 1u : 0u;
  }
  return acc;
}

template <int WG, int S>
struct Seg16to32Smem {
  static constexpr int NW = WG / 64;
  static constexpr uint32_t SEGW = 8u * WG * S;
  static constexpr uint32_t PAD = 16;
  static constexpr uint32_t LIM = PAD + SEGW;
  static constexpr uint32_t DUMP = LIM + 8;
  static constexpr uint32_t SSZ = DUMP + 20;
  uint32_t stage[SSZ];
  uint32_t wtot[NW * (S / 2)];
  uint32_t halo[S * NW];
  unsigned long long seg_base;
  unsigned long long werr;
  uint32_t bounds[2];
};

// UTF-16 (L.be: big-endian words) -> UTF-32: validation by the surrogate sequencing
// check of section 7.4 (analyze16 / locate16); a BMP word is its code point and a pair
// is emitted once, at its low surrogate, as 0x10000 + (high - 0xD800) * 1024 +
// (low - 0xDC00) (section 2.1).  A pair whose high surrogate ends the previous chunk is
// emitted by this chunk.
template <int WG, int S>
__global__ void __launch_bounds__(WG) k_u16_to_u32(Launch L) {
  typedef Seg16to32Smem<WG, S> M;
  __shared__ __attribute__((aligned(16))) M sm;
  constexpr int NW = M::NW;
  constexpr uint32_t TW = 8u * WG;
  constexpr uint32_t SEGW = M::SEGW;
  constexpr uint32_t PAD = M::PAD, LIM = M::LIM, DUMP = M::DUMP;
  const uint64_t seg = blockIdx.x;
  uint32_t x[S][4];
  load_seg16<WG, S>(L, seg, x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t epoch = cur_epoch(L.ws);
  const uint64_t s0 = seg * SEGW;
  const uint64_t q00 = s0 + 8ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const bool segfull = s0 >= lo && s0 + SEGW <= hi;

  const uint32_t wp_seg = (threadIdx.x == 0) ? (load16_prev(L, s0) << 16) : 0u;
  uint32_t c[S];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * TW;
    c[k] = count16_chars(x[k], q0, lo, hi, segfull || (q0 >= lo && q0 + 8 <= hi));
  }
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < S; ++k) sm.halo[k * NW + wid] = x[k][3];
  }
  if (threadIdx.x == 0) sm.werr = NO_ERR;
  uint32_t off[S];
  const uint32_t seg_total = segment_offsets<WG, S>(c, off, sm.wtot);  // contains a barrier
  if (threadIdx.x == 0) {
    debug_delay(L.dbg, seg);
    publish_aggregate(L.status, seg, seg_total, epoch);
  }

#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * TW;
    const uint32_t hl = (wid > 0) ? sm.halo[k * NW + wid - 1] : (k > 0 ? sm.halo[(k - 1) * NW + NW - 1] : wp_seg);
    const uint32_t wp = wave_shr1(x[k][3], hl) >> 16;  // the word before the chunk
    const bool full = segfull || (q0 >= lo && q0 + 8 <= hi);
    uint32_t len[8], cnt;
    bool det;
    if (full) analyze16<true>(x[k], wp, q0, lo, hi, len, cnt, det);
    else analyze16<false>(x[k], wp, q0, lo, hi, len, cnt, det);
    const uint32_t idx = PAD + off[k] - (is_hi(wp) ? 1u : 0u);
    const bool fits = idx + 8 <= LIM;
    uint32_t* pw = sm.stage + (fits ? idx : DUMP);
    uint32_t* const dump = sm.stage + DUMP;
    uint32_t prev = wp;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t w = (x[k][j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
      const bool in = full || (q0 + j >= lo && q0 + j < hi);
      const uint32_t cp = is_lo(w) ? 0x10000u + ((prev - 0xD800u) << 10) + (w - 0xDC00u) : w;
      const uint32_t bit = (in && !is_hi(w)) ? 1u : 0u;
      *(bit ? pw : dump) = cp;
      pw += bit;
      prev = w;
    }
    if (k == 0 && threadIdx.x == 0) sm.bounds[0] = idx;
    if (k == S - 1 && threadIdx.x == WG - 1) sm.bounds[1] = fits ? (uint32_t)(pw - sm.stage) : LIM;
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)L.mis;
      if (before(p0 - 1, sm.werr)) {
        const uint16_t* in16 = reinterpret_cast<const uint16_t*>(L.base) + L.mis;
        const uint64_t e = locate16(in16, L.n, p0 - 1, p0 + 8, L.be != 0);
        if (e != NO_ERR) atomicMin(&sm.werr, (unsigned long long)e);
      }
    }
  }
  if (wid == 0) {
    const uint64_t b = lookback_wave(L.status, seg, seg_total, epoch, L.ws, [&](uint64_t j) {
      return wave_segment_sum(j, SEGW, 8, [&](uint64_t q) {
        uint32_t xx[4];
        load16(L, q, xx);
        return (uint64_t)count16_chars(xx, q, lo, hi, false);
      });
    });
    if (lane == 0) sm.seg_base = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) report_err(L.err, sm.werr);
  const uint32_t st0 = sm.bounds[0];
  uint32_t st1 = sm.bounds[1];
  st1 = st1 < st0 ? st0 : (st1 > LIM ? LIM : st1);
  const int64_t g = (int64_t)sm.seg_base + (int64_t)st0 - (int64_t)PAD;
  store_span<uint32_t>(sm.stage, st0, st1 - st0, reinterpret_cast<uint32_t*>(L.out), (uint64_t)g, L.cap,
                       threadIdx.x, WG);
}

// Result of a UTF-16 -> UTF-32 launch: the characters of the valid prefix (words that
// are not low surrogates before the error), or the total against cap.
template <int WG>
__global__ void __launch_bounds__(WG) k_fin_u16u32(Launch L) {
  __shared__ unsigned long long lds[WG / 64 + 2];
  constexpr uint64_t TW = 8ull * WG;
  const uint64_t err = ld_agent(L.err);
  const bool fault = ld_fault(L.ws) != 0;
  uint64_t written = 0;
  if (!fault && err != NO_ERR) {
    const uint64_t qoff = err + L.mis;
    const uint64_t seg = qoff / L.seg_units;
    uint32_t acc = 0;
    for (uint64_t q0b = seg * L.seg_units; q0b < qoff; q0b += TW) {
      const uint64_t q0 = q0b + 8ull * threadIdx.x;
      uint32_t x[4];
      load16(L, q0, x);
      acc += count16_chars(x, q0, L.mis, qoff, false);
    }
    const uint64_t s = block_sum_u64<WG>(acc, lds);
    written = (seg ? tile_inclusive(L.status, seg - 1) : 0) + s;
  }
  __syncthreads();  // every wave has read err and fault before thread 0 resets them
  if (threadIdx.x == 0) {
    const uint64_t tot = tile_inclusive(L.status, L.ntiles - 1);
    if (fault) write_result(L.result, ST_DEVICE, 0, 0);
    else if (err != NO_ERR) write_result(L.result, ST_SURROGATE, err, written);
    else if (tot > L.cap) write_result(L.result, ST_OUTPUT_TOO_SMALL, tot, 0);
    else write_result(L.result, ST_OK, tot, tot);
    reset_ws(L.ws);
  }
}

// Validation of UTF-32: every unit on its own; the workgroup's first invalid unit in LDS.
template <int WG>
__global__ void __launch_bounds__(WG) k_validate32(Launch L) {
  constexpr uint64_t TU = 4ull * WG;
  __shared__ unsigned long long werr;
  const uint64_t q00 = (uint64_t)blockIdx.x * L.seg * TU + 4ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  if (threadIdx.x == 0) werr = NO_ERR;
  __syncthreads();
  for (uint32_t s = 0; s < L.seg; ++s) {
    const uint64_t q0 = q00 + s * TU;
    uint32_t x[4], fb;
    load32(L, q0, x);
    count32(x, q0, lo, hi, q0 >= lo && q0 + 4 <= hi, &fb);
    if (fb < 4) {
      const uint64_t e = q0 + fb - lo;
      if (before((int64_t)e, werr)) atomicMin(&werr, (unsigned long long)e);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) report_err(L.err, werr);
}

__global__ void k_fin_validate32(Launch L) {
  if (threadIdx.x == 0) {
    const uint64_t err = ld_agent(L.err);
    if (ld_fault(L.ws)) {
      write_result(L.result, ST_DEVICE, 0, 0);
    } else if (err != NO_ERR) {
      const uint32_t u = reinterpret_cast<const uint32_t*>(L.base)[L.mis + err];
      write_result(L.result, (u >= 0xD800u && u <= 0xDFFFu) ? ST_SURROGATE : ST_TOO_LARGE, err, err);
    } else {
      write_result(L.result, ST_OK, L.n, L.n);
    }
    reset_ws(L.ws);
  }
}

}  // namespace utfx_dev
