// utfx_device.hpp -- device-side building blocks for the gfx950 transcoding kernels.
//
// Layout conventions used throughout:
//   * A workgroup owns one tile of T = 16 * WG input bytes; every thread owns one
//     16-byte chunk (four dwords, little-endian: byte 0 of the chunk is the low byte
//     of dword 0).  Tiles are counted over "grid positions": the input pointer is
//     rounded down to 16 bytes and grid position q is the byte at base + q, so that
//     every full chunk is one aligned 16-byte load.  Logical input position
//     p = q - mis, where mis = in - base.
//   * Per-byte flags are kept in SWAR form: bit 7 of each byte of a dword.
//   * The tile scan publishes one 64-bit status word per tile for a decoupled
//     look-back (Merrill & Garland): epoch (25 bits) | flag (2 bits) | value (37 bits).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace utfx_dev {

constexpr uint32_t HI = 0x80808080u;
constexpr uint64_t NO_ERR = ~0ull;

constexpr int VAL_BITS = 37;
constexpr uint64_t VAL_MASK = (1ull << VAL_BITS) - 1;
constexpr uint64_t FLAG_AGG = 1;  // tile aggregate available
constexpr uint64_t FLAG_PFX = 2;  // inclusive prefix available
constexpr uint32_t EPOCH_BITS = 25;
constexpr uint32_t EPOCH_MASK = (1u << EPOCH_BITS) - 1;
constexpr uint32_t SPIN_LIMIT = 1u << 22;  // look-back watchdog (iterations of s_sleep)
// Look-back status words sit one per 128-byte line: the words that concurrent
// look-backs poll then spread over many memory channels instead of a few lines.
constexpr uint64_t STATUS_STRIDE = 16;

// Whether a window starting at input position p (may be negative) begins before the
// error offset e (NO_ERR: no error, so every window does).
__device__ __forceinline__ bool before(int64_t p, uint64_t e) { return e == NO_ERR || p < (int64_t)e; }


// Device workspace header (one per context).  The finalisation kernel that ends every
// call resets err and acc and advances the epoch, so a launch always starts from the
// same state without any memset.
struct WsHeader {
  unsigned long long spare0;
  unsigned long long spare1;
  unsigned long long err;       // smallest error offset found (NO_ERR = none)
  unsigned long long acc;       // length-query sum
  uint32_t epoch;               // launch epoch carried by status words
  uint32_t fault;               // sticky: bit 0 = look-back watchdog fired
  unsigned long long pad[3];
};

// Everything a single-buffer kernel needs; passed by value.
struct Launch {
  const uint8_t* base;  // input rounded down to 16 bytes
  uint64_t mis;         // input - base, in input units
  uint64_t n;           // input units
  void* out;            // output (UTF-16 or UTF-8)
  uint64_t cap;         // output units
  WsHeader* ws;                 // epoch and fault flag of the launch
  unsigned long long* err;      // smallest error offset found (NO_ERR = none)
  unsigned long long* status;
  void* result;         // utfx_result* (device)
  uint64_t ntiles;      // workgroups = segments
  uint64_t seg_units;   // input units per segment
  uint32_t seg;         // tiles (one 16-byte chunk per thread) per segment
  uint32_t wg;          // threads per workgroup of the main kernel
  uint32_t be;          // UTF-16 side is big-endian: input words (UTF-16 -> UTF-8) or
                        // output words (UTF-8 -> UTF-16) have their bytes swapped
  uint32_t dbg;         // look-back delay injection (debug_delay); 0 = off
};

// Swaps the bytes of both 16-bit halves (UTF-16BE <-> UTF-16LE code units).
__device__ __forceinline__ uint32_t bswap16x2(uint32_t v) { return __builtin_amdgcn_perm(v, v, 0x02030001u); }
__device__ __forceinline__ uint32_t bswap16(uint32_t w) { return ((w & 0xFFu) << 8) | ((w >> 8) & 0xFFu); }

// Result record layout (matches utfx_result in utfx.h).
struct Result {
  int32_t status;
  uint32_t reserved;
  uint64_t count;
  uint64_t written;
};

enum : int32_t {
  ST_OK = 0,
  ST_STRAY_CONT = 1,
  ST_MISSING_CONT = 2,
  ST_OVERLONG = 3,
  ST_TOO_LARGE = 4,
  ST_SURROGATE = 5,
  ST_BAD_BYTE = 6,
  ST_OUTPUT_TOO_SMALL = 16,
  ST_INVALID_ARG = 17,
  ST_DEVICE = 18
};

// ---------------------------------------------------------------- bit primitives

// v_alignbyte_b32: ({hi, lo} >> 8*s)[31:0]
__device__ __forceinline__ uint32_t abyte(uint32_t hi, uint32_t lo, uint32_t s) {
  return __builtin_amdgcn_alignbyte(hi, lo, s);
}
// v_perm_b32: byte select from {a (bytes 4..7), b (bytes 0..3)}; 8..11 replicate the
// sign of byte 1/3/5/7, 12 gives 0x00, 13..15 give 0xFF.
__device__ __forceinline__ uint32_t perm(uint32_t a, uint32_t b, uint32_t sel) {
  return __builtin_amdgcn_perm(a, b, sel);
}
// 0xFF in every byte whose bit 7 is set, 0x00 elsewhere (two instructions).
__device__ __forceinline__ uint32_t bytemask(uint32_t f) { return perm(f, f << 8, 0x0B090A08u); }
// 16-bit lane masks for byte positions (0,1) and (2,3) of a flag dword.
__device__ __forceinline__ uint32_t lanemask_lo(uint32_t f) { return perm(f, f << 8, 0x0A0A0808u); }
__device__ __forceinline__ uint32_t lanemask_hi(uint32_t f) { return perm(f, f << 8, 0x0B0B0909u); }
// zero-extend bytes (0,1) or (2,3) of a dword into two 16-bit lanes
__device__ __forceinline__ uint32_t zx_lo(uint32_t v) { return perm(0u, v, 0x0C010C00u); }
__device__ __forceinline__ uint32_t zx_hi(uint32_t v) { return perm(0u, v, 0x0C030C02u); }

// a + byte SEL of b in one instruction (an SDWA operand select).  Written out because
// the compiler extracts the byte with a separate shift and mask.
template <int SEL>
__device__ __forceinline__ uint32_t add_byte(uint32_t a, uint32_t b) {
  static_assert(SEL >= 0 && SEL < 4, "byte select");
  uint32_t r;
  if constexpr (SEL == 0)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (SEL == 1)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
        : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (SEL == 2)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
        : "=v"(r) : "v"(a), "v"(b));
  else
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
        : "=v"(r) : "v"(a), "v"(b));
  return r;
}

typedef unsigned short us2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ us2 as_us2(uint32_t v) { return __builtin_bit_cast(us2, v); }
__device__ __forceinline__ uint32_t as_u32(us2 v) { return __builtin_bit_cast(uint32_t, v); }
// 1 in each nonzero 16-bit lane of x, 0 in each zero lane: one v_pk_min_u16 against
// (1, 1).  Written out because the compiler turns min(x, 1) into a compare and a
// select per lane.
__device__ __forceinline__ uint32_t pk_nz(uint32_t x) {
  uint32_t r;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(x), "s"(0x00010001u));
  return r;
}

// lane-wise a*m + c (mod 2^16), one v_pk_mad_u16
__device__ __forceinline__ uint32_t pk_mad(uint32_t a, uint16_t m, uint32_t c) {
  us2 r = as_us2(a) * (us2)(m) + as_us2(c);
  return as_u32(r);
}

// ---------------------------------------------------------------- memory-model helpers

__device__ __forceinline__ unsigned long long ld_agent(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reports a workgroup's first error e (NO_ERR: none) to the launch's minimum.  Atomics
// on one word serialise at the memory side (tens of ns each), so a workgroup reads the
// word first and only lowers it when its error is smaller; with dense errors, most
// workgroups find a smaller one already there.
__device__ __forceinline__ void report_err(unsigned long long* err, uint64_t e) {
  if (e != NO_ERR && e < ld_agent(err)) atomicMin(err, (unsigned long long)e);
}

// ---------------------------------------------------------------- scans

// Inclusive scan over a wave64 with DPP row shifts and row broadcasts (GFX9 forms):
// after row_shr 1/2/4/8 every row of 16 lanes holds its own scan; row_bcast:15 adds
// row 0's total to row 1 and row 2's to row 3; row_bcast:31 adds the first 32 lanes'
// total to lanes 32..63.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// Exclusive scan of one 32-bit value per thread over the workgroup; `total` gets the
// workgroup sum.  scratch holds WG/64 words.  Contains one barrier; the caller must
// pass another barrier before scratch is written again.
template <int WG>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t& total, uint32_t* scratch) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const uint32_t x = wave_incl_scan(v);
  if (lane == 63) scratch[wid] = x;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) {
    uint32_t s = scratch[w];
    before += (w < wid) ? s : 0u;
    tot += s;
  }
  total = tot;
  return before + x - v;
}

template <int WG>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, unsigned long long* scratch) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  uint64_t tot = 0;
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) tot += scratch[w];
  __syncthreads();
  return tot;
}

template <int WG>
__device__ __forceinline__ uint64_t block_min_u64(uint64_t v, unsigned long long* scratch) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint64_t o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  uint64_t m = NO_ERR;
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) m = scratch[w] < m ? scratch[w] : m;
  __syncthreads();
  return m;
}

// Publishes a tile's aggregate (tile 0 publishes its inclusive prefix directly).
__device__ __forceinline__ void publish_aggregate(unsigned long long* status, uint64_t tile, uint64_t agg,
                                                  uint32_t epoch) {
  const unsigned long long tag = (unsigned long long)(epoch & EPOCH_MASK) << (VAL_BITS + 2);
  st_agent(&status[tile * STATUS_STRIDE], tag | ((tile == 0 ? FLAG_PFX : FLAG_AGG) << VAL_BITS) | agg);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Aggregate of segment `seg` recomputed by the calling wave from the input: the sum of
// chunk_count(q0) over the segment's chunks [seg * seg_units, (seg + 1) * seg_units),
// chunk_units units apart (the same chunks and masks the segment's own workgroup
// counted).  Returns the same value in every lane.
template <class F>
__device__ __forceinline__ uint64_t wave_segment_sum(uint64_t seg, uint64_t seg_units, uint32_t chunk_units,
                                                     const F& chunk_count) {
  const uint32_t lane = threadIdx.x & 63;
  uint64_t acc = 0;
  const uint64_t end = (seg + 1) * seg_units;
  for (uint64_t q0 = seg * seg_units + (uint64_t)lane * chunk_units; q0 < end; q0 += 64ull * chunk_units)
    acc += chunk_count(q0);
  return wave_sum_u64(acc);
}

// Polls of one look-back window before the waiting wave stops relying on its
// predecessors' workgroups and computes the nearest missing aggregate itself; after it
// has done so once, it waits only LB_PATIENCE_AFTER polls for the next.
constexpr uint32_t LB_PATIENCE = 64;
constexpr uint32_t LB_PATIENCE_AFTER = 4;

// Decoupled look-back (Merrill & Garland), run by one whole wave after the tile has
// published its aggregate.  Each round loads the status words of the 128 nearest
// unaccounted predecessors (2 per lane, lane 0 nearest) in one coalesced access; if
// every one of them up to the nearest inclusive prefix is ready, their values are
// summed and the walk ends at that prefix (or continues 128 tiles further back).
// Then the tile's own inclusive prefix is published.  Returns the exclusive prefix
// (same value in every lane).
//
// Every wait ends whatever order the hardware runs workgroups in: a predecessor that
// has not published after LB_PATIENCE polls gets its aggregate from agg_of(index) (a
// whole-wave call that recomputes it from the input, e.g. with wave_segment_sum), so
// the walk never depends on another workgroup being resident.  Tile 0's aggregate is
// also its inclusive prefix.  The watchdog stays as a guard against a broken
// invariant and reports through ws->fault.
constexpr int LB_PER_LANE = 2;
template <class AggOf>
__device__ __forceinline__ uint64_t lookback_wave(unsigned long long* status, uint64_t tile, uint64_t agg,
                                                  uint32_t epoch, WsHeader* ws, const AggOf& agg_of) {
  const int lane = threadIdx.x & 63;
  const unsigned long long tag = (unsigned long long)(epoch & EPOCH_MASK) << (VAL_BITS + 2);
  if (tile == 0) return 0;
  uint64_t excl = 0;
  int64_t top = (int64_t)tile - 1;  // nearest predecessor not yet accounted for
  uint32_t spins = 0;
  uint32_t patience = LB_PATIENCE;
  // aggregates this wave computed for the words of its lane in the current window
  bool fx[LB_PER_LANE];
  uint64_t fv[LB_PER_LANE];
#pragma unroll
  for (int j = 0; j < LB_PER_LANE; ++j) {
    fx[j] = false;
    fv[j] = 0;
  }
  while (true) {
    unsigned long long s[LB_PER_LANE];
#pragma unroll
    for (int j = 0; j < LB_PER_LANE; ++j) {
      const int64_t idx = top - (LB_PER_LANE * lane + j);
      s[j] = (idx >= 0) ? ld_agent(&status[idx * STATUS_STRIDE]) : (tag | (FLAG_PFX << VAL_BITS));
      if (fx[j]) s[j] = tag | ((idx == 0 ? FLAG_PFX : FLAG_AGG) << VAL_BITS) | fv[j];
    }
    bool ok[LB_PER_LANE];
    int lane_first = LB_PER_LANE;  // first inclusive prefix among this lane's words
#pragma unroll
    for (int j = LB_PER_LANE - 1; j >= 0; --j) {
      ok[j] = (s[j] >> (VAL_BITS + 2)) == (epoch & EPOCH_MASK) && ((s[j] >> VAL_BITS) & 3) != 0;
      if (ok[j] && ((s[j] >> VAL_BITS) & 3) == FLAG_PFX) lane_first = j;
    }
    const unsigned long long pm = __ballot(lane_first < LB_PER_LANE);
    const int F = pm ? __builtin_ctzll(pm) : 64;  // lane holding the nearest prefix
    // the first word of this lane that is needed (at or before the nearest prefix) and
    // not ready (LB_PER_LANE: none)
    int miss = LB_PER_LANE;
#pragma unroll
    for (int j = LB_PER_LANE - 1; j >= 0; --j) {
      const bool needed = lane < F || (lane == F && j <= lane_first);
      if (needed && !ok[j]) miss = j;
    }
    const unsigned long long mm = __ballot(miss < LB_PER_LANE);
    if (mm) {
      ++spins;
      if (spins >= patience) {
        // compute the nearest missing aggregate here instead of waiting for it
        const int L0 = __builtin_ctzll(mm);
        const int j0 = __shfl(miss, L0, 64);
        const int64_t idx = top - (LB_PER_LANE * L0 + j0);
        const uint64_t v = agg_of((uint64_t)idx);
#pragma unroll
        for (int j = 0; j < LB_PER_LANE; ++j) {
          if (lane == L0 && j == j0) {
            fx[j] = true;
            fv[j] = v;
          }
        }
        patience = LB_PATIENCE_AFTER;
        spins = 0;
        continue;
      }
      if (spins > SPIN_LIMIT) {
        if (lane == 0) atomicOr(&ws->fault, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(4);
      continue;
    }
    uint64_t v = 0;
#pragma unroll
    for (int j = 0; j < LB_PER_LANE; ++j) {
      const bool take = (lane < F) || (lane == F && j <= lane_first);
      v += take ? (uint64_t)(s[j] & VAL_MASK) : 0;
    }
    excl += wave_sum_u64(v);
    if (F < 64) break;
    top -= 64 * LB_PER_LANE;
    spins = 0;
#pragma unroll
    for (int j = 0; j < LB_PER_LANE; ++j) fx[j] = false;
  }
  if (lane == 0) st_agent(&status[tile * STATUS_STRIDE], tag | (FLAG_PFX << VAL_BITS) | (excl + agg));
  return excl;
}

// Debug mode (look-back delay injection): holds back the publication of one segment in
// sixteen, chosen by a hash of its index, by a pseudo-random number of s_sleep(127)
// rounds below 64 * dbg (about 3.4 us each), so that look-backs meet late and missing
// predecessors.  dbg = 0 (the default) skips it.
__device__ __forceinline__ void debug_delay(uint32_t dbg, uint64_t seg) {
  if (dbg == 0) return;
  uint32_t h = (uint32_t)seg * 0x9E3779B1u + (uint32_t)(seg >> 32);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  if ((h & 15u) != 0) return;
  const uint32_t n = (h >> 4) % (64u * dbg);
  for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(127);
}

// Inclusive prefix of a finished tile (valid after every tile of the launch is done).
__device__ __forceinline__ uint64_t tile_inclusive(unsigned long long* status, uint64_t tile) {
  return ld_agent(&status[tile * STATUS_STRIDE]) & VAL_MASK;
}

}  // namespace utfx_dev
