// utfx_transcode.hpp -- single-read validating transcode kernels for gfx950.
//
// A workgroup owns one segment of S tiles (a tile is one 16-byte chunk per thread) and
// reads it from HBM exactly once, into registers:
//   phase A  every chunk's output length by the per-unit length formula (the length
//            query of section 7.5; for valid input it is exact, and each character's
//            units are counted at its first unit), a packed wave scan per pair of
//            tiles, and the segment's total published for the decoupled look-back;
//   phase B  per chunk: classify, validate, decode / encode, and scatter the units
//            into an LDS stage holding the whole segment's output; then wave 0 runs
//            the look-back, by when its predecessors have usually published;
//   store    one barrier, then coalesced 16-byte stores of the stage at the
//            segment's global offset.
// The chunk offsets come from the length formula, where a character is counted at
// its lead; UTF-8 -> UTF-16 emits a character's words at its last bytes (the end mask
// of section 6.1), so a chunk's first emitted word lies below the formula offset by
// the words of characters that start in the 3 bytes before it (its "spill").
#pragma once
#include "utfx_kernels.hpp"

namespace utfx_dev {

// A value the whole wave holds, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// DPP wave_shr:1 -- lane i gets lane i-1's v; lane 0 gets `first`.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v, uint32_t first) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)first, (int)v, 0x138, 0xF, 0xF, false);
}

// Coalesced store of staged output by threads tid = 0..nthr-1: stage element s0 + l
// (0 <= l < total) goes to out[base + l].  16-byte chunks aligned to the destination
// are gathered from the stage with dword reads and a byte funnel shift; elements at or
// beyond cap are never stored.  The stage must hold 16 readable bytes past s0 + total.
// I: the signed type of destination indices (32-bit where base + total and cap are
// known to stay below 2^31).
template <typename T>
struct NoDeduce {
  typedef T type;
};
template <typename U, typename I = int64_t>
__device__ __forceinline__ void store_span(const U* stage, uint32_t s0, uint32_t total, U* out,
                                           typename NoDeduce<I>::type base, typename NoDeduce<I>::type cap,
                                           uint32_t tid, uint32_t nthr, bool swap16 = false) {
  constexpr uint32_t PER = 16 / sizeof(U);
  const uint32_t d = ((uint32_t)((uintptr_t)out / sizeof(U)) + (uint32_t)base) & (PER - 1);
  const uint32_t nch = (d + total + PER - 1) / PER;
  const I g_first = base - (I)d;
  const uint32_t* s32 = reinterpret_cast<const uint32_t*>(stage);
  for (uint32_t k = tid; k < nch; k += nthr) {
    const I g0 = g_first + (I)(k * PER);
    const uint32_t l0 = k * PER;  // chunk covers elements l0 - d .. l0 - d + PER - 1
    if (l0 >= d && l0 + PER <= d + total && g0 + (I)PER <= cap) {
      const uint32_t b0 = (s0 + l0 - d) * sizeof(U);
      const uint32_t w0 = b0 >> 2, sh = b0 & 3;
      const uint32_t v0 = s32[w0], v1 = s32[w0 + 1], v2 = s32[w0 + 2], v3 = s32[w0 + 3], v4 = s32[w0 + 4];
      uint4 o;
      o.x = abyte(v1, v0, sh);
      o.y = abyte(v2, v1, sh);
      o.z = abyte(v3, v2, sh);
      o.w = abyte(v4, v3, sh);
      if (sizeof(U) == 2 && swap16) {
        o.x = bswap16x2(o.x);
        o.y = bswap16x2(o.y);
        o.z = bswap16x2(o.z);
        o.w = bswap16x2(o.w);
      }
      *reinterpret_cast<uint4*>(out + g0) = o;
    } else {
      // An edge chunk: its elements i_lo <= i < i_hi lie in the span and in [0, cap).
      // They are gathered like a whole chunk (s0 >= d, so the window starts inside the
      // stage; it ends within 20 bytes past the span) and stored one by one.
      I a = (I)d - (I)l0, b = (I)d + (I)total - (I)l0;
      a = a > -g0 ? a : -g0;
      b = b < cap - g0 ? b : cap - g0;
      const uint32_t i_lo = a <= 0 ? 0u : (a >= (I)PER ? PER : (uint32_t)a);
      const uint32_t i_hi = b <= 0 ? 0u : (b >= (I)PER ? PER : (uint32_t)b);
      if (i_lo < i_hi) {
        const uint32_t b0 = (s0 + l0 - d) * sizeof(U);
        const uint32_t w0 = b0 >> 2, sh = b0 & 3;
        const uint32_t v0 = s32[w0], v1 = s32[w0 + 1], v2 = s32[w0 + 2], v3 = s32[w0 + 3], v4 = s32[w0 + 4];
        uint32_t o[4] = {abyte(v1, v0, sh), abyte(v2, v1, sh), abyte(v3, v2, sh), abyte(v4, v3, sh)};
        if (sizeof(U) == 2 && swap16) {
#pragma unroll
          for (int j = 0; j < 4; ++j) o[j] = bswap16x2(o[j]);
        }
#pragma unroll
        for (uint32_t i = 0; i < PER; ++i) {
          if (i >= i_lo && i < i_hi) {
            const uint32_t word = o[(i * sizeof(U)) >> 2];
            out[g0 + (I)i] = (U)(word >> (8 * ((i * sizeof(U)) & 3)));
          }
        }
      }
    }
  }
}

// Chunk offsets of a segment from per-chunk counts c[S] (formula units): packed wave
// scans of tile pairs, wave totals through LDS (one barrier), then per chunk the sum of
// the earlier tiles' totals, the earlier waves' totals of its own tile and the
// exclusive scan inside its wave.  Counts must be < 2^16 per tile.  Returns the
// segment total; `wtot` holds NW x S/2 words.
template <int WG, int S>
__device__ __forceinline__ uint32_t segment_offsets(const uint32_t c[S], uint32_t off[S], uint32_t* wtot) {
  constexpr int NW = WG / 64;
  constexpr int P = S / 2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t own[P], inc[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    own[j] = c[2 * j] | (c[2 * j + 1] << 16);
    inc[j] = wave_incl_scan(own[j]);
  }
  if (lane == 63) {
#pragma unroll
    for (int j = 0; j < P; ++j) wtot[wid * P + j] = inc[j];
  }
  __syncthreads();
  uint32_t run = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    uint32_t tot = 0, before = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t t = wtot[w * P + j];
      tot += t;
      before += (w < wid) ? t : 0u;
    }
    const uint32_t ex = before + inc[j] - own[j];  // lane-wise, no carries: each half < 2^16
    off[2 * j] = run + (ex & 0xFFFFu);
    run += tot & 0xFFFFu;
    off[2 * j + 1] = run + (ex >> 16);
    run += tot >> 16;
  }
  return run;
}

// ================================================================ UTF-8 -> UTF-16LE

// Output words of a 16-byte chunk by the length formula: one per byte that is not a
// continuation (10xxxxxx) and one more per byte >= F0 (section 6.2: the 4-byte
// characters become surrogate pairs).  Positions whose mask byte is clear count 0.
__device__ __forceinline__ uint32_t count8(const uint32_t x[4], const uint32_t* m) {
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t v = x[k];
    const uint32_t s1 = v << 1;
    uint32_t nc = (~v | s1) & HI;         // bit 7: not 10xxxxxx
    const uint32_t u = v & s1;            // bit 7: 11xxxxxx, bit 5: xx11xxxx
    uint32_t f = u & (u << 2) & HI;       // bit 7: 1111xxxx
    if (m) {
      nc &= m[k];
      f &= m[k];
    }
    acc += __builtin_popcount(nc) + __builtin_popcount(f);
  }
  return acc;
}

// Words that characters starting in the 3 bytes before a chunk emit inside it: a
// 2-byte lead one back emits at position 0; a lead >= E0 two back emits at 0 and one
// back at 1; a lead >= F0 also emits its low surrogate three back -> 0, two back -> 1,
// one back -> 2.  Cp is the class dword of those bytes (with the >= F0 bits).
__device__ __forceinline__ uint32_t spill8(uint32_t Cp) {
  const uint32_t e = ((Cp >> 24) << 1) | ((Cp >> 16) << 2) | ((Cp >> 8) << 3);
  return __builtin_popcount(e & HI);
}

// One 16-byte chunk of UTF-8 -> UTF-16: classify, validate and decode it, and scatter
// its words into the stage from slot `idx` on (formula offset minus spill, computed
// inside).  x: the chunk; xp: the 4 bytes before it; off: the chunk's formula offset
// relative to the stage's PAD slot.  Returns the slot after the chunk's last word (LIM
// for a chunk that lies past the stage); *det reports a detected error nearby.
template <uint32_t PAD, uint32_t LIM, uint32_t DUMP, typename P = uint64_t>
__device__ __forceinline__ uint32_t chunk_u8_to_u16(const uint32_t x[4], uint32_t xp, bool full, P q0, P lo, P hi,
                                                    uint32_t off, uint16_t* stage,
                                                    uint32_t* first, uint32_t* det_out,
                                                    const uint32_t* mE = nullptr) {
  Chunk8 ch;
#pragma unroll
  for (int i = 0; i < 4; ++i) ch.x[i] = x[i];
  ch.xp = xp;
  uint32_t inE[4], inD[4], E[4], W[8], cnt, det;
  if (!full) {
    // [lo, hi) (the caller's masks when it has them) and [lo, hi]: the same plus the
    // byte at hi
    if (mE) {
#pragma unroll
      for (int k = 0; k < 4; ++k) inE[k] = mE[k];
    } else {
      range_masks(q0, lo, hi, inE);
    }
    typedef typename std::make_signed<P>::type SP;
    const SP t = (SP)hi - (SP)q0;
    const uint32_t tt = (t >= 0 && t < 16) ? (uint32_t)t : 16u;
#pragma unroll
    for (int k = 0; k < 4; ++k) inD[k] = inE[k] | ((tt >> 2) == (uint32_t)k ? 0xFFu << (8 * (tt & 3)) : 0u);
  }
  const int cls = classify8(ch);
  process8_any<true>(cls, full, ch, inE, inD, E, cnt, det, W);
  uint32_t idx = PAD + off - spill8(ch.Cp);
  *first = idx;
  // Scatter.  A non-emitting position writes a placeholder at the slot of the next
  // emit, which that emit overwrites: inside a valid prefix at most two positions in a
  // row do not emit, so only the last two positions can lack a later emit in the chunk,
  // and those write only real words.  Positions outside the input (a chunk at an end)
  // emit nothing: before the input they are followed by the chunk's first emit, and
  // after it every later chunk is outside too; a chunk with no emit at all writes to the
  // dump area.  Past the first error every slot is at or beyond the valid prefix's
  // length, and a chunk whose slots would leave the stage is past it and writes to the
  // dump area.  The byte address of each write is the previous one plus 2 when the
  // previous position emitted: B holds those steps per byte, one add of a byte field
  // each.
  const bool fits = idx + 16 <= LIM;
  const bool any = full || (E[0] | E[1] | E[2] | E[3]) != 0;
  char* const sb = reinterpret_cast<char*>(stage);
  uint16_t* const dump = stage + DUMP;
  uint32_t a = (fits && any) ? 2u * idx : 2u * DUMP;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const uint32_t B = (E[kk] >> 6) & 0x02020202u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = 4 * kk + i;
      const uint32_t pair = W[2 * kk + (i >> 1)];
      const uint16_t word = (uint16_t)((i & 1) ? (pair >> 16) : (pair & 0xFFFFu));
      if (e < 14) {
        *reinterpret_cast<uint16_t*>(sb + a) = word;
      } else {
        const uint32_t bit = (E[kk] >> (8 * i + 7)) & 1u;
        *(bit ? reinterpret_cast<uint16_t*>(sb + a) : dump) = word;
      }
      if (i == 0) a = add_byte<0>(a, B);
      else if (i == 1) a = add_byte<1>(a, B);
      else if (i == 2) a = add_byte<2>(a, B);
      else a = add_byte<3>(a, B);
    }
  }
  idx = !fits ? LIM : (any ? a / 2u : idx);
  *det_out = det;
  return idx;
}

// LDS of one UTF-8 -> UTF-16 segment: the stage holds the segment's output words.
template <int WG, int S>
struct Seg8Smem {
  static constexpr int NW = WG / 64;
  static constexpr uint32_t SEGB = 16u * WG * S;
  static constexpr uint32_t PAD = 16;             // stage slots below the segment's formula offset
  static constexpr uint32_t LIM = PAD + SEGB;     // a valid chunk ends at or below this slot
  static constexpr uint32_t DUMP = LIM + 16;      // 16 slots for writes that must not land
  static constexpr uint32_t SSZ = DUMP + 16;
  uint16_t stage[SSZ];
  uint32_t wtot[NW * (S / 2)];
  uint32_t halo[S * NW];
  unsigned long long seg_base;
  unsigned long long werr;  // first error found by this workgroup
  uint32_t bounds[2];
};

// Loads segment `seg` of a UTF-8 buffer: chunk k of thread t is the 16 bytes at grid
// position seg * SEGB + 16 * (k * WG + t); bytes outside the input read as 0.
template <int WG, int S>
__device__ __forceinline__ void load_seg8(const Launch& L, uint64_t seg, uint32_t (&x)[S][4]) {
  constexpr uint32_t T = 16u * WG;
  const uint64_t s0 = seg * (uint64_t)(T * S);
  const uint64_t q00 = s0 + 16ull * threadIdx.x;
  if (s0 >= L.mis && s0 + T * S <= L.mis + L.n) {
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const uint4 v = *reinterpret_cast<const uint4*>(L.base + q00 + (uint64_t)k * T);
      x[k][0] = v.x; x[k][1] = v.y; x[k][2] = v.z; x[k][3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < S; ++k) load8(L, q00 + (uint64_t)k * T, x[k]);
  }
}

// One segment of a UTF-8 -> UTF-16LE transcode (segment `seg` of the buffer L, loaded
// into x).
//
// Errors: a flagged chunk is located only while it could still lower the workgroup's
// minimum, which is kept in LDS; at the end one thread reports it (report_err), so
// that dense errors do not serialise every lane on the launch's shared word.
template <int WG, int S>
__device__ __forceinline__ void seg_u8_to_u16(const Launch& L, uint64_t seg, Seg8Smem<WG, S>& sm,
                                              const uint32_t (&x)[S][4]) {
  typedef Seg8Smem<WG, S> M;
  constexpr int NW = M::NW;
  constexpr uint32_t T = 16u * WG;
  constexpr uint32_t SEGB = M::SEGB;
  constexpr uint32_t PAD = M::PAD, LIM = M::LIM, DUMP = M::DUMP;
  uint16_t* const stage = sm.stage;
  uint32_t* const wtot = sm.wtot;
  uint32_t* const halo = sm.halo;
  uint32_t* const bounds = sm.bounds;

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t epoch = cur_epoch(L.ws);
  const uint64_t s0 = seg * SEGB;
  const uint64_t q00 = s0 + 16ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const bool segfull = s0 >= lo && s0 + SEGB <= hi;

  // ---- phase A: the segment is in x (loaded by the caller); count, scan
  const uint32_t xp_seg = (threadIdx.x == 0) ? load8_prev(L, s0) : 0u;
  uint32_t c[S];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * T;
    if (segfull || (q0 >= lo && q0 + 16 <= hi)) {
      c[k] = count8(x[k], nullptr);
    } else {
      uint32_t m[4];
      range_masks(q0, lo, hi, m);
      c[k] = count8(x[k], m);
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < S; ++k) halo[k * NW + wid] = x[k][3];
  }
  if (threadIdx.x == 0) sm.werr = NO_ERR;
  uint32_t off[S];
  const uint32_t seg_total = segment_offsets<WG, S>(c, off, wtot);  // contains a barrier

  if (threadIdx.x == 0) {
    debug_delay(L.dbg, seg);
    publish_aggregate(L.status, seg, seg_total, epoch);
  }

  // ---- phase B: per chunk, validate + decode + scatter into the stage
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * T;
    const uint32_t hl = (wid > 0) ? halo[k * NW + wid - 1] : (k > 0 ? halo[(k - 1) * NW + NW - 1] : xp_seg);
    uint32_t first, det;
    const bool full = segfull || (q0 >= lo && q0 + 16 <= hi);
    const uint32_t idx = chunk_u8_to_u16<PAD, LIM, DUMP>(x[k], wave_shr1(x[k][3], hl), full, q0, lo, hi, off[k],
                                                         stage, &first, &det);
    if (k == 0 && threadIdx.x == 0) bounds[0] = first;
    if (k == S - 1 && threadIdx.x == WG - 1) bounds[1] = idx;
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)L.mis;
      if (before(p0 - 3, sm.werr)) {
        const uint64_t e = locate8(L.base + L.mis, L.n, p0 - 3, p0 + 16);
        if (e != NO_ERR) atomicMin(&sm.werr, (unsigned long long)e);
      }
    }
  }
  if (wid == 0) {
    // the look-back runs after the wave's own work, when predecessors are likely done
    const uint64_t b = lookback_wave(L.status, seg, seg_total, epoch, L.ws, [&](uint64_t j) {
      return wave_segment_sum(j, SEGB, 16, [&](uint64_t q) {
        uint32_t xx[4], mm[4];
        load8(L, q, xx);
        range_masks(q, lo, hi, mm);
        return (uint64_t)count8(xx, mm);
      });
    });
    if (lane == 0) sm.seg_base = b;
  }
  __syncthreads();

  if (threadIdx.x == 0) report_err(L.err, sm.werr);

  // ---- store the segment's output
  const uint32_t st0 = bounds[0];
  uint32_t st1 = bounds[1];
  st1 = st1 < st0 ? st0 : (st1 > LIM ? LIM : st1);
  const int64_t g = (int64_t)sm.seg_base + (int64_t)st0 - (int64_t)PAD;
  store_span<uint16_t>(stage, st0, st1 - st0, reinterpret_cast<uint16_t*>(L.out), (uint64_t)g, L.cap,
                       threadIdx.x, WG, L.be != 0);
}

template <int WG, int S>
__global__ void __launch_bounds__(WG) k_u8_to_u16(Launch L) {
  __shared__ __attribute__((aligned(16))) Seg8Smem<WG, S> sm;
  uint32_t x[S][4];
  load_seg8<WG, S>(L, blockIdx.x, x);
  seg_u8_to_u16<WG, S>(L, blockIdx.x, sm, x);
}

// Words of the valid prefix in[0:off]: the exclusive prefix of off's segment plus the
// length formula over the segment's positions before off (exact there, because every
// character before the first error is complete).
template <int WG>
__device__ uint64_t prefix_words8(const Launch& L, uint64_t off, uint64_t seg_units, unsigned long long* lds) {
  constexpr uint64_t T = 16ull * WG;
  const uint64_t qoff = off + L.mis;
  const uint64_t seg = qoff / seg_units;
  uint32_t acc = 0;
  uint32_t x[4], m[4];
  for (uint64_t q0b = seg * seg_units; q0b < qoff; q0b += T) {
    const uint64_t q0 = q0b + 16ull * threadIdx.x;
    load8(L, q0, x);
    range_masks(q0, L.mis, qoff, m);
    acc += count8(x, m);
  }
  const uint64_t s = block_sum_u64<WG>(acc, lds);
  const uint64_t before = seg ? tile_inclusive(L.status, seg - 1) : 0;
  return before + s;
}

// Result of a UTF-8 -> UTF-16LE launch: error kind and the words of the valid prefix,
// or the total (checked against cap).
template <int WG>
__global__ void __launch_bounds__(WG) k_fin_u8u16(Launch L) {
  __shared__ unsigned long long lds[WG / 64 + 2];
  const uint64_t err = ld_agent(L.err);
  const bool fault = ld_fault(L.ws) != 0;
  uint64_t written = 0;
  if (!fault && err != NO_ERR) written = prefix_words8<WG>(L, err, L.seg_units, lds);
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

// ================================================================ UTF-16LE -> UTF-8

typedef short ss2 __attribute__((ext_vector_type(2)));

// Output bytes of the two words of X (16-bit lanes): 1 below U+0080, 2 below U+0800,
// 2 for each half of a surrogate pair, else 3 (section 7.3).
__device__ __forceinline__ uint32_t pk_len16s(uint32_t X) {
  const us2 w = as_us2(X);
  return pk_nz(as_u32(w >> (us2)(7))) + pk_nz(as_u32(w >> (us2)(11))) + pk_nz((X & 0xF800F800u) ^ 0xD800D800u);
}

// Lane-wise unpaired-surrogate detection for the words of X, with P holding each
// word's predecessor: a word is flagged when "is a low surrogate" differs from "the
// word before is a high surrogate" (sections 2.1 and 7.4).
__device__ __forceinline__ uint32_t pk_pair_err(uint32_t X, uint32_t P) {
  const uint32_t a = pk_nz((X & 0xFC00FC00u) ^ 0xDC00DC00u);  // 0: a low surrogate
  const uint32_t b = pk_nz((P & 0xFC00FC00u) ^ 0xD800D800u);  // 0: after a high surrogate
  return a ^ b;  // nonzero lanes: unpaired
}

// UTF-8 bytes of the two words of X with surrogates (little-endian in a dword each),
// P = each word's predecessor, c_lo / c_hi = their lengths.  Figure 1(a) forms: the
// 3-byte form [E0|w>>12, 80|(w>>6 & 3F), 80|(w & 3F)]; the 2-byte form [C0|w>>6,
// 80|(w & 3F)].  A high surrogate emits the first two bytes of its 4-byte character,
// which depend on it alone: with u = w - 0xD7C0 (the code point >> 10, section 7.2)
// they are [F0|u>>8, 80|(u>>2 & 3F)], i.e. the 2-byte form of u>>2 with the tag
// raised from C0 to F0.  A low surrogate emits the last two, [80|(h & 3)<<4|(w>>6 &
// F), 80|(w & 3F)] with h its high surrogate: the 2-byte form's bytes with the tag
// bits 5..4 replaced by h's bits 1..0.
__device__ __forceinline__ void pk_enc16s(uint32_t X, uint32_t P, uint32_t c_lo, uint32_t c_hi, uint32_t& v_lo,
                                          uint32_t& v_hi) {
  const us2 w = as_us2(X);
  const uint32_t ns = pk_nz((X & 0xF800F800u) ^ 0xD800D800u);      // 1: not a surrogate
  const uint32_t mS = as_u32(as_us2(ns) - (us2)(1));                // 0xFFFF: surrogate
  const uint32_t b10 = as_u32(__builtin_bit_cast(us2, __builtin_bit_cast(ss2, X << 5) >> (ss2)(15)));
  const uint32_t mH = mS & ~b10, mL = mS & b10;                     // high / low surrogate lanes
  const uint32_t D = as_u32((w - (us2)(0xD7C0)) >> (us2)(2));
  const uint32_t Wp = (mH & D) | (~mH & X);
  const uint32_t p0 = as_u32(w >> (us2)(12)) | 0x00E000E0u;
  const uint32_t p1 = (as_u32(as_us2(Wp) >> (us2)(6)) & 0x003F003Fu) | 0x00800080u;
  const uint32_t p2 = (Wp & 0x003F003Fu) | 0x00800080u;
  const uint32_t tag = (mL & ~(P << 4) & 0x00300030u) | (~mL & 0x00400040u) | (mH & 0x00300030u);
  const uint32_t l2 = p1 ^ tag;
  const uint32_t q12 = p1 | (p2 << 8);
  const uint32_t q2 = l2 | (p2 << 8);
  const uint32_t t3l = perm(q12, p0, 0x0C050400u), t3h = perm(q12, p0, 0x0C070602u);
  const uint32_t t2l = perm(q2, 0u, 0x0C0C0504u), t2h = perm(q2, 0u, 0x0C0C0706u);
  v_lo = c_lo == 3 ? t3l : (c_lo == 2 ? t2l : (X & 0xFFFFu));
  v_hi = c_hi == 3 ? t3h : (c_hi == 2 ? t2h : (X >> 16));
}

// 16-bit lane masks (0xFFFF) of the chunk words a <= j < b (0 <= a, b <= 8), as four
// dwords of two words each; the per-lane bias of 0x8000 keeps the subtractions from
// borrowing across lanes (see byte_masks_ab).
__device__ __forceinline__ void word_masks_ab(uint32_t a, uint32_t b, uint32_t m[4]) {
  const uint32_t A = a * 0x00010001u, B = (b * 0x00010001u) | 0x80008000u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t idx = 0x00010000u + 0x00020002u * k;
    const uint32_t in = ((idx | 0x80008000u) - A) & (B - (idx + 0x00010001u)) & 0x80008000u;
    m[k] = (in >> 15) * 0xFFFFu;
  }
}

// Word masks of the chunk's word positions q0 + j in [lo, hi).
__device__ __forceinline__ void word_masks(uint64_t q0, uint64_t lo, uint64_t hi, uint32_t m[4]) {
  const int64_t a64 = (int64_t)lo - (int64_t)q0, b64 = (int64_t)hi - (int64_t)q0;
  const uint32_t a = a64 <= 0 ? 0u : (a64 >= 8 ? 8u : (uint32_t)a64);
  const uint32_t b = b64 <= 0 ? 0u : (b64 >= 8 ? 8u : (uint32_t)b64);
  word_masks_ab(a, b, m);
}

// word_masks in 32-bit arithmetic, for positions below 2^31.
__device__ __forceinline__ void word_masks32(uint32_t q0, uint32_t lo, uint32_t hi, uint32_t m[4]) {
  const int32_t a32 = (int32_t)lo - (int32_t)q0, b32 = (int32_t)hi - (int32_t)q0;
  const uint32_t a = a32 <= 0 ? 0u : (a32 >= 8 ? 8u : (uint32_t)a32);
  const uint32_t b = b32 <= 0 ? 0u : (b32 >= 8 ? 8u : (uint32_t)b32);
  word_masks_ab(a, b, m);
}

// Output bytes of a chunk of 8 words; with word masks, words outside count 0.
__device__ __forceinline__ uint32_t count16(const uint32_t x[4], const uint32_t* m) {
  uint32_t l = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) l += m ? (pk_len16s(x[k]) & m[k]) : pk_len16s(x[k]);
  return (l & 0xFFFFu) + (l >> 16);
}

// Writes the c (0..3) bytes of v at p.  With own_only false, a word with c >= 1
// writes all three bytes (the spare ones are overwritten by later words of the
// chunk); otherwise, and for c = 0, the bytes that are not its own go to the dump
// slot, so there are no branches.
__device__ __forceinline__ void put3(uint8_t* p, uint32_t v, uint32_t c, bool own_only, uint8_t* dump) {
  *(c >= 1 ? p : dump) = (uint8_t)v;
  *((c >= 2 || (!own_only && c >= 1)) ? p + 1 : dump) = (uint8_t)(v >> 8);
  *((c >= 3 || (!own_only && c >= 1)) ? p + 2 : dump) = (uint8_t)(v >> 16);
}
// The same for a word known to have c >= 1 that may write spare bytes.
__device__ __forceinline__ void put3_all(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v;
  p[1] = (uint8_t)(v >> 8);
  p[2] = (uint8_t)(v >> 16);
}

// One chunk of 8 words of UTF-16 -> UTF-8: validate, encode and scatter its bytes to
// st (the chunk's first output byte).  x: the chunk with words outside the input
// zeroed; xprev: the dword before the chunk (its high half is the word before, zero
// before the input); m: word masks of the positions inside the input, or null when
// all are.  Zeroed words are neither surrogate, so they flag nothing, and their
// lengths are masked to 0.  Returns whether an error was detected nearby.
template <bool MASKED>
__device__ __forceinline__ bool chunk_u16_to_u8_t(const uint32_t x[4], uint32_t xprev, const uint32_t* m,
                                                  uint8_t* st, uint8_t* dump) {
  const uint32_t wp = xprev >> 16;
  bool det = false;
  uint32_t o = 0;
  // a word of an unmasked chunk has c >= 1, so words 0..5 may write all three bytes
  auto put = [&](uint32_t v, uint32_t c, int kk) {
    if (!MASKED && kk < 3) put3_all(st + o, v);
    else put3(st + o, v, c, kk == 3, dump);
    o += c;
  };
  if (!__any(any_surrogate(x, wp))) {
    // no surrogate anywhere in the wave's chunks: lengths 1..3, nothing to validate.
    // Each word writes three bytes at its offset; the spare ones are overwritten by
    // the following words (each adds at least one byte), except for the last two
    // words of the chunk, which write only their own bytes.
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const uint32_t l = MASKED ? (pk_len16(x[kk]) & m[kk]) : pk_len16(x[kk]);
      const uint32_t cl = l & 0xFFFFu, chh = l >> 16;
      uint32_t vl, vh;
      pk_enc16(x[kk], cl, chh, vl, vh);
      put(vl, cl, kk);
      put(vh, chh, kk);
    }
  } else {
    uint32_t d = 0, prevd = xprev;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const uint32_t X = x[kk];
      const uint32_t P = abyte(X, prevd, 2);  // each word's predecessor
      d |= pk_pair_err(X, P);
      const uint32_t l = MASKED ? (pk_len16s(X) & m[kk]) : pk_len16s(X);
      const uint32_t cl = l & 0xFFFFu, chh = l >> 16;
      uint32_t vl, vh;
      pk_enc16s(X, P, cl, chh, vl, vh);
      put(vl, cl, kk);
      put(vh, chh, kk);
      prevd = X;
    }
    det = d != 0;
  }
  return det;
}

__device__ __forceinline__ bool chunk_u16_to_u8(const uint32_t x[4], uint32_t xprev, const uint32_t* m,
                                                uint8_t* st, uint8_t* dump) {
  return m ? chunk_u16_to_u8_t<true>(x, xprev, m, st, dump) : chunk_u16_to_u8_t<false>(x, xprev, m, st, dump);
}

// LDS of one UTF-16 -> UTF-8 segment: the stage holds the segment's output bytes.
template <int WG, int S>
struct Seg16Smem {
  static constexpr int NW = WG / 64;
  static constexpr uint32_t SEGW = 8u * WG * S;
  static constexpr uint32_t PAD = 16;
  static constexpr uint32_t DUMP = PAD + 3 * SEGW + 32;  // slot for writes that must not land
  static constexpr uint32_t SSZ = DUMP + 16;
  uint8_t stage[SSZ];
  uint32_t wtot[NW * (S / 2)];
  uint32_t halo[S * NW];
  unsigned long long seg_base;
  unsigned long long werr;  // first error found by this workgroup
};

// Loads segment `seg` of a UTF-16 buffer (words outside the input read as 0).
template <int WG, int S>
__device__ __forceinline__ void load_seg16(const Launch& L, uint64_t seg, uint32_t (&x)[S][4]) {
  constexpr uint32_t TW = 8u * WG;
  const uint64_t s0 = seg * (uint64_t)(TW * S);
  const uint64_t q00 = s0 + 8ull * threadIdx.x;
  const uint16_t* in16 = reinterpret_cast<const uint16_t*>(L.base);
  if (s0 >= L.mis && s0 + TW * S <= L.mis + L.n) {
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const uint4 v = *reinterpret_cast<const uint4*>(in16 + q00 + (uint64_t)k * TW);
      x[k][0] = v.x; x[k][1] = v.y; x[k][2] = v.z; x[k][3] = v.w;
    }
    if (L.be) {
#pragma unroll
      for (int k = 0; k < S; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[k][j] = bswap16x2(x[k][j]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < S; ++k) load16(L, q00 + (uint64_t)k * TW, x[k]);
  }
}

// One segment of a UTF-16LE -> UTF-8 transcode (loaded into x; errors as in
// seg_u8_to_u16).
template <int WG, int S>
__device__ __forceinline__ void seg_u16_to_u8(const Launch& L, uint64_t seg, Seg16Smem<WG, S>& sm,
                                              const uint32_t (&x)[S][4]) {
  typedef Seg16Smem<WG, S> M;
  constexpr int NW = M::NW;
  constexpr uint32_t TW = 8u * WG;      // words per tile
  constexpr uint32_t SEGW = M::SEGW;
  constexpr uint32_t PAD = M::PAD, DUMP = M::DUMP;
  uint8_t* const stage = sm.stage;
  uint32_t* const wtot = sm.wtot;
  uint32_t* const halo = sm.halo;

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t epoch = cur_epoch(L.ws);
  const uint64_t s0 = seg * SEGW;
  const uint64_t q00 = s0 + 8ull * threadIdx.x;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const bool segfull = s0 >= lo && s0 + SEGW <= hi;
  const uint16_t* in16 = reinterpret_cast<const uint16_t*>(L.base);

  // ---- phase A: the segment is in x (loaded by the caller)
  // the word before the segment, in the high half (the layout of a chunk's last dword)
  const uint32_t xp_seg = (threadIdx.x == 0) ? (load16_prev(L, s0) << 16) : 0u;
  uint32_t c[S];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * TW;
    if (segfull || (q0 >= lo && q0 + 8 <= hi)) {
      c[k] = count16(x[k], nullptr);
    } else {
      uint32_t m[4];
      word_masks(q0, lo, hi, m);
      c[k] = count16(x[k], m);
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < S; ++k) halo[k * NW + wid] = x[k][3];
  }
  if (threadIdx.x == 0) sm.werr = NO_ERR;
  uint32_t off[S];
  const uint32_t seg_total = segment_offsets<WG, S>(c, off, wtot);

  if (threadIdx.x == 0) {
    debug_delay(L.dbg, seg);
    publish_aggregate(L.status, seg, seg_total, epoch);
  }

  // ---- phase B
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const uint64_t q0 = q00 + (uint64_t)k * TW;
    const uint32_t hl = (wid > 0) ? halo[k * NW + wid - 1] : (k > 0 ? halo[(k - 1) * NW + NW - 1] : xp_seg);
    const uint32_t xprev = wave_shr1(x[k][3], hl);  // high half: the word before the chunk
    bool det;
    if (segfull) {
      det = chunk_u16_to_u8(x[k], xprev, nullptr, stage + PAD + off[k], stage + DUMP);
    } else {
      uint32_t m[4];
      word_masks(q0, lo, hi, m);
      det = chunk_u16_to_u8(x[k], xprev, m, stage + PAD + off[k], stage + DUMP);
    }
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)L.mis;
      if (before(p0 - 1, sm.werr)) {
        const uint16_t* in = in16 + L.mis;
        const uint64_t e = locate16(in, L.n, p0 - 1, p0 + 8, L.be != 0);
        if (e != NO_ERR) atomicMin(&sm.werr, (unsigned long long)e);
      }
    }
  }
  if (wid == 0) {
    // the look-back runs after the wave's own work, when predecessors are likely done
    const uint64_t b = lookback_wave(L.status, seg, seg_total, epoch, L.ws, [&](uint64_t j) {
      return wave_segment_sum(j, SEGW, 8, [&](uint64_t q) {
        uint32_t xx[4], mm[4];
        load16(L, q, xx);
        word_masks(q, lo, hi, mm);
        return (uint64_t)count16(xx, mm);
      });
    });
    if (lane == 0) sm.seg_base = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) report_err(L.err, sm.werr);
  store_span<uint8_t>(stage, PAD, seg_total, reinterpret_cast<uint8_t*>(L.out), sm.seg_base, L.cap, threadIdx.x,
                      WG);
}

// Segments of up to four tiles fit in 80 VGPRs: six waves per SIMD, so that the LDS
// (not the registers) bounds the workgroups per CU.
template <int WG, int S>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(S <= 4 ? 6 : 1))) k_u16_to_u8(Launch L) {
  __shared__ __attribute__((aligned(16))) Seg16Smem<WG, S> sm;
  uint32_t x[S][4];
  load_seg16<WG, S>(L, blockIdx.x, x);
  seg_u16_to_u8<WG, S>(L, blockIdx.x, sm, x);
}

template <int WG>
__device__ uint64_t prefix_bytes16(const Launch& L, uint64_t off, uint64_t seg_units, unsigned long long* lds) {
  constexpr uint64_t TW = 8ull * WG;
  const uint64_t qoff = off + L.mis;
  const uint64_t seg = qoff / seg_units;
  uint32_t acc = 0;
  uint32_t x[4];
  for (uint64_t q0b = seg * seg_units; q0b < qoff; q0b += TW) {
    const uint64_t q0 = q0b + 8ull * threadIdx.x;
    uint32_t m[4];
    load16(L, q0, x);
    word_masks(q0, L.mis, qoff, m);
    acc += count16(x, m);
  }
  const uint64_t s = block_sum_u64<WG>(acc, lds);
  const uint64_t before = seg ? tile_inclusive(L.status, seg - 1) : 0;
  return before + s;
}

template <int WG>
__global__ void __launch_bounds__(WG) k_fin_u16u8(Launch L) {
  __shared__ unsigned long long lds[WG / 64 + 2];
  const uint64_t err = ld_agent(L.err);
  const bool fault = ld_fault(L.ws) != 0;
  uint64_t written = 0;
  if (!fault && err != NO_ERR) written = prefix_bytes16<WG>(L, err, L.seg_units, lds);
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

}  // namespace utfx_dev
