// utfx_batch.hpp -- many independent strings in one call (the batched path).
//
// Every string (item) gets the result the single-buffer call would give on its bytes.
// Kernels, in stream order:
//   k_batch_begin  advance the batch epoch; clear the segment totals, the list counts,
//                  the length sum and the fault flag (one thread, so the call needs no
//                  memset and can be captured into a graph);
//   k_batch_plan   per item: check its descriptor (an invalid one gets its result
//                  here) and, for a large item (more than small_max input units), count
//                  its segments; exclusive scans of the counts over items, one per
//                  direction (workgroup scan + decoupled look-back across workgroups);
//                  each large item writes the segment -> item map of its segments and
//                  enters the large-item list; each tiny item enters its direction's
//                  tiny-item list; every other item enters the list of its length
//                  class (by the number of 1 KiB steps it takes);
//   k_batch_tiny   four tiny items (at most TINY8 bytes / TINY16 words) per wave, one per
//                  16-lane row: a row holds the whole string in one step;
//   k_batch_small  one wave per item of the length-class lists, longest class first:
//                  the wave walks the string 1 KiB (512 words) at a time carrying the
//                  output offset (no look-back, no barrier) and writes the item's result;
//   k_batch_large  one persistent launch per direction: each workgroup takes every G-th
//                  segment of the large items (G = its grid) and runs the single-buffer
//                  segment code on it, the look-back ending at the item's first segment;
//   k_batch_fin    one workgroup per large item: the result from its segments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdio.h>

#include <type_traits>

#include "utfx.h"
#include "utfx_transcode.hpp"

namespace utfx_dev {

struct BItem {  // utfx_item
  uint64_t in_off, in_len, out_off, out_cap;
  uint32_t dir, pad;
};

// Items up to this many input units are transcoded by one wave (the default of the
// tunable BatchArgs::small_max).
constexpr uint64_t SMALL_MAX = 16384;
// Length classes of the wave-walked items, by the steps (1 KiB of UTF-8 or 512 words of
// UTF-16) a wave takes: class 0 = more than 8 steps, 1 = 5..8, 2 = 3..4, 3 = 1..2.
constexpr int NCLS = 4;
// Geometry of the large-item segments (workgroup size, tiles per segment per direction).
// Geometry of the large-item segments: 512-thread workgroups of bs tiles (2 or 4,
// tunable), so bs * 8 KiB of UTF-8 or bs * 4096 words of UTF-16 per segment.
constexpr int BWG = 512;
constexpr int PLAN_WG = 256;
constexpr int PLAN_ITEMS = 4;  // items per plan thread

struct BatchArgs {
  const uint8_t* in;
  uint8_t* out;
  uint64_t in_bytes, out_bytes;      // arena sizes
  const BItem* items;
  Result* results;
  uint64_t n_items;
  // ws: epoch, fault; acc = large items; err = sum of in_len over the valid items;
  // spare1 / pad[1] = segment totals and spare0 / pad[0] = tiny-item counts of the
  // UTF-8 / UTF-16 items
  WsHeader* ws;
  unsigned long long* unit_start;    // n_items: an item's first segment in its direction's numbering
  unsigned long long* item_err;      // n_items: first error of a large item
  unsigned long long* status[2];     // cap_units each: look-back status word per segment (strided)
  uint32_t* unit_item[2];            // cap_units each: item of each segment
  uint32_t* large;                   // n_items: list of large items
  uint32_t* tiny[2];                 // n_items each: list of tiny items per direction
  uint32_t* small[NCLS];             // n_items each: wave-walked items per length class
  unsigned long long* cls_count;     // NCLS: lengths of the small[] lists
  unsigned long long* plan_status[2];  // one status word per plan workgroup and direction (strided)
  uint64_t cap_units;
  uint64_t total_in;                 // the caller's bound on the sum of in_len
  uint32_t rows;                     // tiny items go to k_batch_tiny (large calls only)
  uint64_t small_max;                // items above this many units take segments
  uint32_t bs;                       // tiles per large-item segment (2 or 4)
  uint32_t dbg;                      // look-back delay injection (debug_delay); 0 = off
};

// Whether the plan holds: the items add up to at most the caller's bound, and so
// their segments fit the workspace.
__device__ __forceinline__ bool plan_ok(const BatchArgs& A) {
  return ld_agent(&A.ws->err) <= A.total_in && ld_agent(&A.ws->spare1) <= A.cap_units &&
         ld_agent(&A.ws->pad[1]) <= A.cap_units;
}

__device__ __forceinline__ unsigned long long* total_of(WsHeader* ws, int dir) {
  return dir ? &ws->pad[1] : &ws->spare1;
}
__device__ __forceinline__ unsigned long long* ntiny_of(WsHeader* ws, int dir) {
  return dir ? &ws->pad[0] : &ws->spare0;
}

// Tiny items: with the start's misalignment (< 16 bytes) and the end position, the
// whole string lies in one 16-lane row step (256 bytes / 128 words).
constexpr uint64_t TINY8 = 240, TINY16 = 120;
__device__ __forceinline__ bool item_tiny(const BItem& it) { return it.in_len <= (it.dir ? TINY16 : TINY8); }

__device__ __forceinline__ bool item_ok(const BatchArgs& A, const BItem& it) {
  if (it.dir > 1 || it.in_len > (1ull << 35) || it.out_cap > (3ull << 35)) return false;
  const uint64_t iu = it.dir ? 2 : 1, ou = it.dir ? 1 : 2;
  if (it.in_off > A.in_bytes || it.in_len * iu > A.in_bytes - it.in_off) return false;
  if (it.out_off > A.out_bytes || it.out_cap * ou > A.out_bytes - it.out_off) return false;
  if (it.dir == 1 && (((uintptr_t)(A.in + it.in_off)) & 1)) return false;   // UTF-16 input
  if (it.dir == 0 && (((uintptr_t)(A.out + it.out_off)) & 1)) return false;  // UTF-16 output
  return true;
}

__device__ __forceinline__ uint64_t item_units(const BatchArgs& A, const BItem& it) {
  const uint32_t unit = it.dir ? 2u : 1u;
  const uint64_t mis = (((uintptr_t)(A.in + it.in_off)) & 15) / unit;
  const uint64_t seg = (it.dir ? 8ull : 16ull) * BWG * A.bs;
  return (mis + it.in_len + 1 + seg - 1) / seg;
}

// The single-buffer launch description of a large item.
__device__ __forceinline__ Launch item_launch(const BatchArgs& A, const BItem& it, uint64_t i) {
  Launch L;
  const uint32_t unit = it.dir ? 2u : 1u;
  const uintptr_t a = (uintptr_t)(A.in + it.in_off);
  L.base = reinterpret_cast<const uint8_t*>(a & ~(uintptr_t)15);
  L.mis = (a & 15) / unit;
  L.n = it.in_len;
  L.out = A.out + it.out_off;
  L.cap = it.out_cap;
  L.ws = A.ws;
  L.err = A.item_err + i;
  L.status = A.status[it.dir] + A.unit_start[i] * STATUS_STRIDE;
  L.result = A.results + i;
  L.ntiles = item_units(A, it);
  L.seg_units = (it.dir ? 8ull : 16ull) * BWG * A.bs;
  L.seg = A.bs;
  L.wg = BWG;
  L.be = 0;
  L.dbg = A.dbg;
  return L;
}

__global__ void k_batch_begin(WsHeader* ws, unsigned long long* cls_count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NCLS; ++c) st_agent(&cls_count[c], 0);
    const uint32_t ep = __hip_atomic_load(&ws->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ws->epoch, (ep + 1) & EPOCH_MASK, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st_agent(&ws->spare0, 0);
    st_agent(&ws->spare1, 0);
    st_agent(&ws->pad[0], 0);
    st_agent(&ws->pad[1], 0);
    st_agent(&ws->acc, 0);
    st_agent(&ws->err, 0);
    __hip_atomic_store(&ws->fault, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Length class of a wave-walked item: the wave takes floor((mis + n) / step) + 1 steps.
__device__ __forceinline__ uint32_t item_class(const BatchArgs& A, const BItem& it) {
  const uint32_t unit = it.dir ? 2u : 1u;
  const uint64_t mis = (((uintptr_t)(A.in + it.in_off)) & 15) / unit;
  const uint64_t steps = (mis + it.in_len) / (it.dir ? 512 : 1024) + 1;
  return steps > 8 ? 0u : (steps > 4 ? 1u : (steps > 2 ? 2u : 3u));
}

__global__ void __launch_bounds__(PLAN_WG) k_batch_plan(BatchArgs A) {
  __shared__ uint32_t scr[6][PLAN_WG / 64];
  __shared__ unsigned long long cbase[NCLS];
  __shared__ unsigned long long pfx[2], lbase[3];
  __shared__ unsigned long long sum_scr[PLAN_WG / 64 + 2];
  // PLAN_ITEMS consecutive items per thread
  const uint64_t i0 = ((uint64_t)blockIdx.x * PLAN_WG + threadIdx.x) * PLAN_ITEMS;
  uint32_t units[PLAN_ITEMS], dir[PLAN_ITEMS], tsum[2] = {0, 0}, tiny = 0, ntiny[2] = {0, 0};
  uint32_t cls = 0, ncls[NCLS] = {0, 0, 0, 0};  // cls: 3 bits per item (class + 1, 0 = none)
  uint64_t len = 0;
  BItem its[PLAN_ITEMS];  // all of the thread's descriptors are loaded before any is used
#pragma unroll
  for (int j = 0; j < PLAN_ITEMS; ++j) {
    if (i0 + j < A.n_items) its[j] = A.items[i0 + j];
  }
#pragma unroll
  for (int j = 0; j < PLAN_ITEMS; ++j) {
    units[j] = 0;
    dir[j] = 0;
    const uint64_t i = i0 + j;
    if (i < A.n_items) {
      const BItem it = its[j];
      if (item_ok(A, it)) {
        len += it.in_len;
        if (it.in_len > A.small_max) {
          units[j] = (uint32_t)item_units(A, it);
          dir[j] = it.dir;
          tsum[it.dir] += units[j];
        } else if (A.rows && item_tiny(it)) {
          tiny |= (1u + it.dir) << (2 * j);  // 1: UTF-8, 2: UTF-16
          ntiny[it.dir]++;
        } else {
          const uint32_t c = item_class(A, it);
          cls |= (c + 1u) << (3 * j);
          ncls[c]++;
        }
      } else {
        write_result(A.results + i, ST_INVALID_ARG, 0, 0);
      }
    }
  }
  const uint64_t len_sum = block_sum_u64<PLAN_WG>(len, sum_scr);
  if (threadIdx.x == 0 && len_sum) atomicAdd(&A.ws->err, (unsigned long long)len_sum);
  uint32_t total[2], local[2];
  local[0] = block_excl_scan<PLAN_WG>(tsum[0], total[0], scr[0]);
  local[1] = block_excl_scan<PLAN_WG>(tsum[1], total[1], scr[1]);
  const uint32_t epoch = cur_epoch(A.ws);
  if (threadIdx.x < 128) {
    // one wave per direction, so that the two look-backs overlap
    const int d = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) {
      debug_delay(A.dbg, blockIdx.x);
      publish_aggregate(A.plan_status[d], blockIdx.x, total[d], epoch);
    }
    // a plan workgroup's aggregate, recomputed from its items if it is late
    const uint64_t b = lookback_wave(A.plan_status[d], blockIdx.x, total[d], epoch, A.ws, [&](uint64_t blk) {
      const uint64_t a0 = blk * (uint64_t)(PLAN_WG * PLAN_ITEMS);
      const uint64_t a1 = a0 + PLAN_WG * PLAN_ITEMS < A.n_items ? a0 + PLAN_WG * PLAN_ITEMS : A.n_items;
      uint64_t acc = 0;
      for (uint64_t i = a0 + (threadIdx.x & 63); i < a1; i += 64) {
        const BItem it = A.items[i];
        if (item_ok(A, it) && it.in_len > A.small_max && (int)it.dir == d) acc += item_units(A, it);
      }
      return wave_sum_u64(acc);
    });
    if ((threadIdx.x & 63) == 0) pfx[d] = b;
  }
  // slots in the lists of large, tiny and wave-walked items (their order is free): the
  // workgroup's counts are scanned and one lane per list takes the list's range with
  // one atomicAdd
  uint32_t nlarge = 0;
#pragma unroll
  for (int j = 0; j < PLAN_ITEMS; ++j) nlarge += units[j] != 0;
  uint32_t ctot[4];
  const uint32_t c0 = block_excl_scan<PLAN_WG>(nlarge | (ntiny[0] << 16), ctot[0], scr[2]);
  const uint32_t c1 = block_excl_scan<PLAN_WG>(ntiny[1], ctot[1], scr[3]);
  const uint32_t c2 = block_excl_scan<PLAN_WG>(ncls[0] | (ncls[1] << 16), ctot[2], scr[4]);
  const uint32_t c3 = block_excl_scan<PLAN_WG>(ncls[2] | (ncls[3] << 16), ctot[3], scr[5]);
  if (threadIdx.x < 3 + NCLS) {
    // one list per lane, so that the atomics are in flight together
    const int q = (int)threadIdx.x;
    const uint32_t want[3 + NCLS] = {ctot[0] & 0xFFFFu, ctot[0] >> 16, ctot[1],        ctot[2] & 0xFFFFu,
                                     ctot[2] >> 16,     ctot[3] & 0xFFFFu, ctot[3] >> 16};
    unsigned long long* const ctr = q == 0 ? &A.ws->acc
                                    : q < 3 ? ntiny_of(A.ws, q - 1)
                                            : &A.cls_count[q - 3];
    const unsigned long long v = want[q] ? atomicAdd(ctr, (unsigned long long)want[q]) : 0ull;
    if (q < 3) lbase[q] = v;
    else cbase[q - 3] = v;
  }
  __syncthreads();
  unsigned long long slot = lbase[0] + (c0 & 0xFFFFu);
  unsigned long long tslot[2] = {lbase[1] + (c0 >> 16), lbase[2] + c1};
  unsigned long long cslot[NCLS] = {cbase[0] + (c2 & 0xFFFFu), cbase[1] + (c2 >> 16), cbase[2] + (c3 & 0xFFFFu),
                                    cbase[3] + (c3 >> 16)};
  uint64_t run[2] = {pfx[0] + local[0], pfx[1] + local[1]};
#pragma unroll
  for (int j = 0; j < PLAN_ITEMS; ++j) {
    const uint64_t i = i0 + j;
    if (i >= A.n_items) break;
    const uint32_t tj = (tiny >> (2 * j)) & 3u;
    if (tj) A.tiny[tj - 1][tslot[tj - 1]++] = (uint32_t)i;
    const uint32_t cj = (cls >> (3 * j)) & 7u;
#pragma unroll
    for (int q = 0; q < NCLS; ++q) {
      if (cj == (uint32_t)q + 1u) A.small[q][cslot[q]++] = (uint32_t)i;
    }
    const int d = (int)dir[j];
    const uint64_t start = run[d];
    A.unit_start[i] = start;
    if (units[j]) {
      A.item_err[i] = NO_ERR;
      A.large[slot++] = (uint32_t)i;
      if (start + units[j] <= A.cap_units)
        for (uint32_t u = 0; u < units[j]; ++u) A.unit_item[d][start + u] = (uint32_t)i;
      run[d] += units[j];
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    st_agent(total_of(A.ws, 0), pfx[0] + total[0]);
    st_agent(total_of(A.ws, 1), pfx[1] + total[1]);
  }
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  return v;
}

// Loads the 16-byte chunk at grid position q0 with the bytes outside the string
// zeroed (m: range_masks of the string).  The aligned 16 bytes are read with one load
// when they lie inside the arena [alo, ahi), else byte by byte; chunks with no byte of
// the string read nothing.
__device__ __forceinline__ void load8_masked(const Launch& L, uint64_t q0, const uint32_t m[4], uintptr_t alo,
                                             uintptr_t ahi, uint32_t x[4]) {
  x[0] = x[1] = x[2] = x[3] = 0;
  if ((m[0] | m[1] | m[2] | m[3]) == 0) return;
  const uintptr_t a = (uintptr_t)(L.base + q0);
  if (a >= alo && a + 16 <= ahi) {
    const uint4 v = *reinterpret_cast<const uint4*>(a);
    x[0] = v.x & m[0]; x[1] = v.y & m[1]; x[2] = v.z & m[2]; x[3] = v.w & m[3];
  } else {
    load8(L, q0, x);
  }
}

// Loads the wave's 1 KiB step at grid position c0 of a UTF-8 string [lo, hi) into x
// (bytes outside the string read as 0) and returns whether every lane's chunk lies
// wholly inside it (wave-uniform).  base: the string's start aligned down to 16 bytes;
// positions are 32-bit (a walked string is far shorter than 2^31 bytes).
__device__ __forceinline__ bool wave_load8(const uint8_t* base, uint32_t c0, uint32_t lo, uint32_t hi,
                                           uintptr_t alo, uintptr_t ahi, uint32_t lane, uint32_t x[4]) {
  const uint32_t q0 = c0 + 16u * lane;
  const bool full = c0 >= lo && c0 + 1024 <= hi;  // every lane's chunk (the same test per lane)
  if (full) {
    const uint4 v = *reinterpret_cast<const uint4*>(base + q0);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else {
    uint32_t m[4];
    range_masks32(q0, lo, hi, m);
    x[0] = x[1] = x[2] = x[3] = 0;
    if ((m[0] | m[1] | m[2] | m[3]) != 0) {
      const uintptr_t a = (uintptr_t)(base + q0);
      if (a >= alo && a + 16 <= ahi) {
        const uint4 v = *reinterpret_cast<const uint4*>(a);
        x[0] = v.x & m[0]; x[1] = v.y & m[1]; x[2] = v.z & m[2]; x[3] = v.w & m[3];
      } else {
        // at an end of the arena: only the string's own bytes are read
#pragma unroll
        for (uint32_t i = 0; i < 16; ++i) {
          const uint32_t q = q0 + i;
          if (q >= lo && q < hi) x[i >> 2] |= (uint32_t)base[q] << (8 * (i & 3));
        }
      }
    }
  }
  return full;
}

// One wave transcodes a UTF-8 string of n bytes (any n; n <= small_max here) 1 KiB at a time; the
// next step's bytes are loaded while the current step is decoded and stored.
// stage: the wave's LDS (WSTAGE bytes); [alo, ahi): the input arena.  A chunk with any
// lane partly outside the string runs the masked path on every lane, so the wave
// never executes both paths.
constexpr uint32_t WSTAGE = 2176;
__device__ __forceinline__ void wave_u8_to_u16(const uint8_t* in, uint64_t n, uint16_t* out, uint64_t cap, uint16_t* stage,
                               Result* res, uintptr_t alo, uintptr_t ahi) {
  constexpr uint32_t PAD = 16, LIM = PAD + 1024, DUMP = LIM + 16;
  static_assert((DUMP + 16) * 2 <= WSTAGE, "wave stage");
  const uint32_t lane = threadIdx.x & 63;
  Launch L = {};
  L.base = reinterpret_cast<const uint8_t*>((uintptr_t)in & ~(uintptr_t)15);
  L.mis = (uintptr_t)in & 15;
  L.n = n;
  // positions, offsets and the capacity in 32 bits: n <= small_max <= 2^18, so every
  // position and output offset of the walk stays below 2^20; the capacity is clamped
  // to 2^30 - 1, which no offset reaches, so that no index difference overflows
  const uint32_t lo = (uint32_t)L.mis, hi = (uint32_t)(L.mis + n);
  const int32_t cap32 = cap > 0x3FFFFFFFull ? 0x3FFFFFFF : (int32_t)cap;
  uint32_t running = 0;  // formula units before the chunk
  uint32_t carry = 0;    // the 4 bytes before the chunk
  uint64_t err = NO_ERR;
  uint32_t xn[4];
  bool fulln = wave_load8(L.base, 0, lo, hi, alo, ahi, lane, xn);
  for (uint32_t c0 = 0; c0 <= hi; c0 += 1024) {
    const uint32_t q0 = c0 + 16u * lane;
    const bool full = fulln;
    uint32_t x[4] = {xn[0], xn[1], xn[2], xn[3]};
    if (c0 + 1024 <= hi) fulln = wave_load8(L.base, c0 + 1024, lo, hi, alo, ahi, lane, xn);
    uint32_t cnt, m[4];
    if (full) {
      cnt = count8(x, nullptr);
    } else {
      range_masks32(q0, lo, hi, m);
      cnt = count8(x, m);
    }
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t tot = __shfl(incl, 63, 64);
    const uint32_t xp = wave_shr1(x[3], carry);
    carry = __shfl(x[3], 63, 64);
    uint32_t first, det;
    const uint32_t end =
        chunk_u8_to_u16<PAD, LIM, DUMP>(x, xp, full, q0, lo, hi, incl - cnt, stage, &first, &det, m);
    const uint32_t st0 = __shfl(first, 0, 64);
    uint32_t st1 = __shfl(end, 63, 64);
    st1 = st1 < st0 ? st0 : (st1 > LIM ? LIM : st1);
    __builtin_amdgcn_wave_barrier();
    store_span<uint16_t, int32_t>(stage, st0, st1 - st0, out, (int32_t)(running + st0 - PAD), cap32, lane, 64);
    __builtin_amdgcn_wave_barrier();
    if (__any(det)) {
      uint64_t e = NO_ERR;
      if (det) {
        const int64_t p0 = (int64_t)q0 - (int64_t)lo;
        e = locate8(in, n, p0 - 3, p0 + 16);
      }
      e = wave_min_u64(e);
      if (e != NO_ERR) {
        err = e;
        break;
      }
    }
    running += tot;
  }
  if (err != NO_ERR) {
    // words of the valid prefix: the length formula over [0, err)
    uint64_t acc = 0;
    for (uint64_t c0 = 0; c0 < L.mis + err; c0 += 1024) {
      const uint64_t q0 = c0 + 16ull * lane;
      uint32_t x[4], m[4];
      load8(L, q0, x);
      range_masks(q0, L.mis, L.mis + err, m);
      acc += count8(x, m);
    }
    acc = wave_sum_u64(acc);
    if (lane == 0) write_result(res, utf8_kind_at(in, n, err), err, acc);
  } else if (lane == 0) {
    if (running > cap) write_result(res, ST_OUTPUT_TOO_SMALL, running, 0);
    else write_result(res, ST_OK, running, running);
  }
}

// Word-masked load of the 8-word chunk at grid position q0 (see load8_masked).
__device__ __forceinline__ void load16_masked(const Launch& L, uint64_t q0, const uint32_t m[4], uintptr_t alo,
                                              uintptr_t ahi, uint32_t x[4]) {
  x[0] = x[1] = x[2] = x[3] = 0;
  if ((m[0] | m[1] | m[2] | m[3]) == 0) return;
  const uintptr_t a = (uintptr_t)(L.base + 2 * q0);
  if (a >= alo && a + 16 <= ahi) {
    const uint4 v = *reinterpret_cast<const uint4*>(a);
    x[0] = v.x & m[0]; x[1] = v.y & m[1]; x[2] = v.z & m[2]; x[3] = v.w & m[3];
  } else {
    load16(L, q0, x);
  }
}

// Loads the wave's 512-word step at grid position c0 of a UTF-16 string [lo, hi) into x
// (words outside the string read as 0); returns whether it lies wholly inside.
__device__ __forceinline__ bool wave_load16(const uint8_t* base, uint32_t c0, uint32_t lo, uint32_t hi,
                                            uintptr_t alo, uintptr_t ahi, uint32_t lane, uint32_t x[4]) {
  const uint32_t q0 = c0 + 8u * lane;
  const bool full = c0 >= lo && c0 + 512 <= hi;  // every lane's chunk (the same test per lane)
  if (full) {
    const uint4 v = *reinterpret_cast<const uint4*>(base + 2 * q0);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else {
    uint32_t m[4];
    word_masks32(q0, lo, hi, m);
    x[0] = x[1] = x[2] = x[3] = 0;
    if ((m[0] | m[1] | m[2] | m[3]) != 0) {
      const uintptr_t a = (uintptr_t)(base + 2 * q0);
      if (a >= alo && a + 16 <= ahi) {
        const uint4 v = *reinterpret_cast<const uint4*>(a);
        x[0] = v.x & m[0]; x[1] = v.y & m[1]; x[2] = v.z & m[2]; x[3] = v.w & m[3];
      } else {
        const uint16_t* w = reinterpret_cast<const uint16_t*>(base);
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
          const uint32_t q = q0 + i;
          if (q >= lo && q < hi) x[i >> 1] |= (uint32_t)w[q] << (16 * (i & 1));
        }
      }
    }
  }
  return full;
}

// One wave transcodes a UTF-16LE string of n words (any n; n <= small_max here) 512 words at a
// time, loading the next step while the current one is encoded and stored.
__device__ __forceinline__ void wave_u16_to_u8(const uint16_t* in, uint64_t n, uint8_t* out, uint64_t cap, uint8_t* stage,
                               Result* res, uintptr_t alo, uintptr_t ahi) {
  constexpr uint32_t PAD = 16, DUMP = PAD + 3 * 512 + 32;
  static_assert(DUMP + 16 <= WSTAGE, "wave stage");
  const uint32_t lane = threadIdx.x & 63;
  Launch L = {};
  L.base = reinterpret_cast<const uint8_t*>((uintptr_t)in & ~(uintptr_t)15);
  L.mis = ((uintptr_t)in & 15) / 2;
  L.n = n;
  // 32-bit positions, offsets and capacity, as in wave_u8_to_u16 (output <= 3n bytes)
  const uint32_t lo = (uint32_t)L.mis, hi = (uint32_t)(L.mis + n);
  const int32_t cap32 = cap > 0x3FFFFFFFull ? 0x3FFFFFFF : (int32_t)cap;
  uint32_t running = 0;
  uint32_t carry = 0;  // high half: the word before the chunk
  uint64_t err = NO_ERR;
  uint32_t xn[4];
  bool fulln = wave_load16(L.base, 0, lo, hi, alo, ahi, lane, xn);
  for (uint32_t c0 = 0; c0 <= hi; c0 += 512) {
    const uint32_t q0 = c0 + 8u * lane;
    const bool full = fulln;
    uint32_t x[4] = {xn[0], xn[1], xn[2], xn[3]};
    if (c0 + 512 <= hi) fulln = wave_load16(L.base, c0 + 512, lo, hi, alo, ahi, lane, xn);
    uint32_t m[4];
    if (!full) word_masks32(q0, lo, hi, m);
    const uint32_t cnt = full ? count16(x, nullptr) : count16(x, m);
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t tot = __shfl(incl, 63, 64);
    const uint32_t xprev = wave_shr1(x[3], carry);
    carry = __shfl(x[3], 63, 64);
    const bool det = full ? chunk_u16_to_u8(x, xprev, nullptr, stage + PAD + (incl - cnt), stage + DUMP)
                          : chunk_u16_to_u8(x, xprev, m, stage + PAD + (incl - cnt), stage + DUMP);
    __builtin_amdgcn_wave_barrier();
    store_span<uint8_t, int32_t>(stage, PAD, tot, out, (int32_t)running, cap32, lane, 64);
    __builtin_amdgcn_wave_barrier();
    if (__any(det)) {
      uint64_t e = NO_ERR;
      if (det) {
        const int64_t p0 = (int64_t)q0 - (int64_t)lo;
        e = locate16(in, n, p0 - 1, p0 + 8);
      }
      e = wave_min_u64(e);
      if (e != NO_ERR) {
        err = e;
        break;
      }
    }
    running += tot;
  }
  if (err != NO_ERR) {
    uint64_t acc = 0;
    for (uint64_t c0 = 0; c0 < L.mis + err; c0 += 512) {
      const uint64_t q0 = c0 + 8ull * lane;
      uint32_t x[4], m[4];
      load16(L, q0, x);
      word_masks(q0, L.mis, L.mis + err, m);
      acc += count16(x, m);
    }
    acc = wave_sum_u64(acc);
    if (lane == 0) write_result(res, ST_SURROGATE, err, acc);
  } else if (lane == 0) {
    if (running > cap) write_result(res, ST_OUTPUT_TOO_SMALL, running, 0);
    else write_result(res, ST_OK, running, running);
  }
}

// ---------------------------------------------------------------- tiny items, by rows

// Inclusive scan over the 16 lanes of each row, and the lane before in the row (0 for
// the row's first lane).
__device__ __forceinline__ uint32_t row_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
  return x;
}
__device__ __forceinline__ uint32_t row_prev(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t row_min_u64(uint64_t v) {
#pragma unroll
  for (int d = 8; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t row_sum_u32(uint32_t v) {
#pragma unroll
  for (int d = 8; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Per row: its item (mine = the row holds one), LDS stage bytes of one row.
constexpr uint32_t TROW = 608;  // >= 2 * (16 + 256 + 32) and 16 + 3 * 128 + 32 + 16

// One step of wave_u8_to_u16 for four strings at once, one per 16-lane row.  The same
// per-chunk code runs on every lane; rows without an item see an empty string.
__device__ __forceinline__ void rows_u8_to_u16(const BatchArgs& A, const BItem& it, bool mine, Result* res,
                                               uint16_t* stage, uintptr_t alo, uintptr_t ahi) {
  constexpr uint32_t PAD = 16, LIM = PAD + 256, DUMP = LIM + 16;
  static_assert((DUMP + 16) * 2 <= TROW, "row stage");
  const uint32_t lane = threadIdx.x & 63, rl = lane & 15, rb = lane & 48;
  const uint8_t* in = A.in + it.in_off;
  Launch L = {};
  L.base = reinterpret_cast<const uint8_t*>((uintptr_t)in & ~(uintptr_t)15);
  L.mis = (uintptr_t)in & 15;
  L.n = mine ? it.in_len : 0;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const uint64_t q0 = 16ull * rl;
  uint32_t x[4], m[4];
  range_masks(q0, lo, hi, m);
  load8_masked(L, q0, m, alo, ahi, x);
  const uint32_t cnt = count8(x, m);
  const uint32_t incl = row_incl_scan(cnt);
  const uint32_t tot = __shfl(incl, rb + 15, 64);
  uint32_t first, det;
  const uint32_t end = chunk_u8_to_u16<PAD, LIM, DUMP>(x, row_prev(x[3]), false, q0, lo, hi, incl - cnt, stage,
                                                       &first, &det, m);
  const uint32_t st0 = __shfl(first, rb, 64);
  uint32_t st1 = __shfl(end, rb + 15, 64);
  st1 = st1 < st0 ? st0 : (st1 > LIM ? LIM : st1);
  __builtin_amdgcn_wave_barrier();
  if (mine)
    store_span<uint16_t>(stage, st0, st1 - st0, reinterpret_cast<uint16_t*>(A.out + it.out_off), st0 - PAD,
                         it.out_cap, rl, 16);
  uint64_t err = NO_ERR;
  if (__any(det)) {
    uint64_t e = NO_ERR;
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)lo;
      e = locate8(in, L.n, p0 - 3, p0 + 16);
    }
    err = row_min_u64(e);
  }
  // words of the valid prefix: the length formula over [0, err)
  uint32_t mp[4];
  range_masks(q0, lo, err == NO_ERR ? hi : lo + err, mp);
  const uint32_t acc = row_sum_u32(count8(x, mp));
  if (mine && rl == 0) {
    if (err != NO_ERR) write_result(res, utf8_kind_at(in, L.n, err), err, acc);
    else if (tot > it.out_cap) write_result(res, ST_OUTPUT_TOO_SMALL, tot, 0);
    else write_result(res, ST_OK, tot, tot);
  }
}

// The same for UTF-16LE -> UTF-8 (one step of wave_u16_to_u8 per row).
__device__ __forceinline__ void rows_u16_to_u8(const BatchArgs& A, const BItem& it, bool mine, Result* res,
                                               uint8_t* stage, uintptr_t alo, uintptr_t ahi) {
  constexpr uint32_t PAD = 16, DUMP = PAD + 3 * 128 + 32;
  static_assert(DUMP + 16 <= TROW, "row stage");
  const uint32_t lane = threadIdx.x & 63, rl = lane & 15, rb = lane & 48;
  const uint16_t* in = reinterpret_cast<const uint16_t*>(A.in + it.in_off);
  Launch L = {};
  L.base = reinterpret_cast<const uint8_t*>((uintptr_t)in & ~(uintptr_t)15);
  L.mis = ((uintptr_t)in & 15) / 2;
  L.n = mine ? it.in_len : 0;
  const uint64_t lo = L.mis, hi = L.mis + L.n;
  const uint64_t q0 = 8ull * rl;
  uint32_t x[4], m[4];
  word_masks(q0, lo, hi, m);
  load16_masked(L, q0, m, alo, ahi, x);
  const uint32_t cnt = count16(x, m);
  const uint32_t incl = row_incl_scan(cnt);
  const uint32_t tot = __shfl(incl, rb + 15, 64);
  const bool det = chunk_u16_to_u8(x, row_prev(x[3]), m, stage + PAD + (incl - cnt), stage + DUMP);
  __builtin_amdgcn_wave_barrier();
  if (mine) store_span<uint8_t>(stage, PAD, tot, A.out + it.out_off, 0, it.out_cap, rl, 16);
  uint64_t err = NO_ERR;
  if (__any(det)) {
    uint64_t e = NO_ERR;
    if (det) {
      const int64_t p0 = (int64_t)q0 - (int64_t)lo;
      e = locate16(in, L.n, p0 - 1, p0 + 8);
    }
    err = row_min_u64(e);
  }
  uint32_t mp[4];
  word_masks(q0, lo, err == NO_ERR ? hi : lo + err, mp);
  const uint32_t acc = row_sum_u32(count16(x, mp));
  if (mine && rl == 0) {
    if (err != NO_ERR) write_result(res, ST_SURROGATE, err, acc);
    else if (tot > it.out_cap) write_result(res, ST_OUTPUT_TOO_SMALL, tot, 0);
    else write_result(res, ST_OK, tot, tot);
  }
}

// Waves [0, W8) take four UTF-8 tiny items each from the UTF-8 list, the next waves four
// UTF-16 items each; waves past both lists exit.
constexpr int TINY_WG = 256;
constexpr uint32_t TINY_ROWS_MIN = 4096;  // items per call from which tiny items use rows
__global__ void __launch_bounds__(TINY_WG) k_batch_tiny(BatchArgs A) {
  constexpr int NW = TINY_WG / 64;
  __shared__ __attribute__((aligned(16))) uint8_t smem[NW * 4 * TROW];
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t lane = threadIdx.x & 63, row = lane >> 4;
  const uint64_t w = (uint64_t)blockIdx.x * NW + wid;
  const uint64_t n8 = ld_agent(ntiny_of(A.ws, 0)), n16 = ld_agent(ntiny_of(A.ws, 1));
  const uint64_t w8 = (n8 + 3) / 4, w16 = (n16 + 3) / 4;
  if (w >= w8 + w16) return;
  const int d = w < w8 ? 0 : 1;  // wave-uniform
  const uint64_t k = 4 * (d ? w - w8 : w) + row;
  const bool mine = k < (d ? n16 : n8);
  const uint32_t i = mine ? A.tiny[d][k] : 0u;
  BItem it = A.items[i];
  Result* res = A.results + i;
  uint8_t* st = smem + (wid * 4 + row) * TROW;
  const uintptr_t alo = (uintptr_t)A.in, ahi = (uintptr_t)(A.in + A.in_bytes);
  if (d == 0) rows_u8_to_u16(A, it, mine, res, reinterpret_cast<uint16_t*>(st), alo, ahi);
  else rows_u16_to_u8(A, it, mine, res, st, alo, ahi);
}

// Persistent over the segments of the large items of one direction: workgroup g takes
// segments g, g + G, g + 2G, ... (G = its grid).  A look-back that waits too long
// recomputes its predecessor's aggregate, so no order of workgroups can stall it.
template <int DIR, int BS>
__global__ void __launch_bounds__(BWG) __attribute__((amdgpu_waves_per_eu(4))) k_batch_large(BatchArgs A) {
  typedef typename std::conditional<DIR == 0, Seg8Smem<BWG, BS>, Seg16Smem<BWG, BS>>::type Smem;
  __shared__ __attribute__((aligned(16))) Smem sm;
  if (!plan_ok(A)) return;
  const uint64_t total = uniform_u64(ld_agent(total_of(A.ws, DIR)));
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const uint32_t i = __builtin_amdgcn_readfirstlane(A.unit_item[DIR][t]);
    const BItem it = A.items[i];
    const Launch L = item_launch(A, it, i);
    const uint64_t seg = t - A.unit_start[i];
    if constexpr (DIR == 0) {
      uint32_t x[BS][4];
      load_seg8<BWG, BS>(L, seg, x);
      seg_u8_to_u16<BWG, BS>(L, seg, sm, x);
    } else {
      uint32_t x[BS][4];
      load_seg16<BWG, BS>(L, seg, x);
      seg_u16_to_u8<BWG, BS>(L, seg, sm, x);
    }
    __syncthreads();  // the stage is reused by the next segment
  }
}

// One wave per wave-walked item, taken from the length-class lists in order, the
// longest class first: the waves of a workgroup get strings of about the same length
// and the longest strings start first.  Waves past the lists' end exit; the list
// lengths are read through the scalar cache, so those waves leave quickly.  (A
// persistent loop over the lists instead needs more than 96 VGPRs and spills.)  At
// most 80 VGPRs: six waves per SIMD, which the walkers' 32-bit positions fit without
// spill (five waves per SIMD measured 2-4 % slower than six).
constexpr int SMALL_WG = 256;
__global__ void __launch_bounds__(SMALL_WG) __attribute__((amdgpu_waves_per_eu(6))) k_batch_small(BatchArgs A) {
  constexpr int NW = SMALL_WG / 64;
  __shared__ __attribute__((aligned(16))) uint8_t smem[NW * WSTAGE];
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint64_t k = (uint64_t)blockIdx.x * NW + wid;
  const unsigned long long* __restrict__ cc = A.cls_count;
  int c = 0;
  for (; c < NCLS; ++c) {
    const uint64_t n = cc[c];
    if (k < n) break;
    k -= n;
  }
  if (c == NCLS) return;
  const uint32_t i = __builtin_amdgcn_readfirstlane(A.small[c][k]);
  const BItem it = A.items[i];
  Result* res = A.results + i;
  uint8_t* st = smem + wid * WSTAGE;
  const uintptr_t alo = (uintptr_t)A.in, ahi = (uintptr_t)(A.in + A.in_bytes);
  if (it.dir == 0)
    wave_u8_to_u16(A.in + it.in_off, it.in_len, reinterpret_cast<uint16_t*>(A.out + it.out_off), it.out_cap,
                   reinterpret_cast<uint16_t*>(st), res, alo, ahi);
  else
    wave_u16_to_u8(reinterpret_cast<const uint16_t*>(A.in + it.in_off), it.in_len, A.out + it.out_off,
                   it.out_cap, st, res, alo, ahi);
}

constexpr int FIN_WG = 256;
__global__ void __launch_bounds__(FIN_WG) k_batch_fin(BatchArgs A) {
  __shared__ unsigned long long lds[FIN_WG / 64 + 2];
  const uint64_t nl = ld_agent(&A.ws->acc);
  const bool over = !plan_ok(A);
  const bool fault = ld_fault(A.ws) != 0;
  for (uint64_t k = blockIdx.x; k < nl; k += gridDim.x) {
    const uint32_t i = A.large[k];
    const BItem it = A.items[i];
    Result* r = A.results + i;
    if (over) {
      if (threadIdx.x == 0) write_result(r, ST_INVALID_ARG, 0, 0);
      continue;
    }
    const Launch L = item_launch(A, it, i);
    const uint64_t err = ld_agent(L.err);
    uint64_t written = 0;
    if (!fault && err != NO_ERR)
      written = it.dir == 0 ? prefix_words8<FIN_WG>(L, err, L.seg_units, lds)
                            : prefix_bytes16<FIN_WG>(L, err, L.seg_units, lds);
    if (threadIdx.x == 0) {
      const uint64_t tot = tile_inclusive(L.status, L.ntiles - 1);
      if (fault) write_result(r, ST_DEVICE, 0, 0);
      else if (err != NO_ERR)
        write_result(r, it.dir == 0 ? utf8_kind_at(L.base + L.mis, L.n, err) : ST_SURROGATE, err, written);
      else if (tot > L.cap) write_result(r, ST_OUTPUT_TOO_SMALL, tot, 0);
      else write_result(r, ST_OK, tot, tot);
    }
  }
}

}  // namespace utfx_dev

// ---------------------------------------------------------------- host side

struct BatchWs {
  void* mem = nullptr;
  utfx_dev::WsHeader* ws = nullptr;
  unsigned long long* unit_start = nullptr;
  unsigned long long* item_err = nullptr;
  unsigned long long* status[2] = {nullptr, nullptr};
  uint32_t* unit_item[2] = {nullptr, nullptr};
  uint32_t* large = nullptr;
  uint32_t* tiny[2] = {nullptr, nullptr};
  uint32_t* small[utfx_dev::NCLS] = {nullptr, nullptr, nullptr, nullptr};
  unsigned long long* cls_count = nullptr;
  unsigned long long* plan_status[2] = {nullptr, nullptr};
  uint64_t cap_items = 0, cap_units = 0;
  uint64_t launches = 0;
  uint64_t gen = 0;  // workspace generation: +1 whenever the old one is freed (a new
                    // allocation may come back at the same address)
};

inline hipError_t batch_ws_init(BatchWs&) { return hipSuccess; }

inline void batch_ws_free(BatchWs& b) {
  if (b.mem) (void)hipFree(b.mem);
  b = BatchWs();
}

// Clears every status word and initialises the header.  Synchronous.
inline hipError_t batch_ws_clear(BatchWs& b, hipStream_t s) {
  const size_t plan_words = (b.cap_items + utfx_dev::PLAN_WG - 1) / utfx_dev::PLAN_WG;  // >= plan blocks
  hipError_t e = hipSuccess;
  for (int d = 0; d < 2 && e == hipSuccess; ++d) {
    e = hipMemsetAsync(b.status[d], 0, b.cap_units * utfx_dev::STATUS_STRIDE * sizeof(unsigned long long), s);
    if (e == hipSuccess) e = hipMemsetAsync(b.plan_status[d], 0, plan_words * utfx_dev::STATUS_STRIDE * sizeof(unsigned long long), s);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(utfx_dev::k_ws_init, dim3(1), dim3(64), 0, s, b.ws);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  b.launches = 0;
  return e;
}

// Sizes the workspace for n_items items and cap_units segments per direction (grows
// by doubling; synchronises the stream when it grows).
inline hipError_t batch_ws_ensure(BatchWs& b, hipStream_t s, uint64_t n_items, uint64_t cap_units) {
  if (n_items <= b.cap_items && cap_units <= b.cap_units) {
    if (b.launches >= (1ull << 24)) return batch_ws_clear(b, s);
    return hipSuccess;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  uint64_t ni = b.cap_items ? b.cap_items : 1024, nu = b.cap_units ? b.cap_units : 4096;
  while (ni < n_items) ni *= 2;
  while (nu < cap_units) nu *= 2;
  if (b.mem) (void)hipFree(b.mem);
  b.mem = nullptr;
  b.gen++;
  const uint64_t plan_words = (ni + utfx_dev::PLAN_WG - 1) / utfx_dev::PLAN_WG;
  auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
  uint64_t o = al(sizeof(utfx_dev::WsHeader));
  const uint64_t o_start = o; o += al(ni * 8);
  const uint64_t o_err = o; o += al(ni * 8);
  const uint64_t o_large = o; o += al(ni * 4);
  const uint64_t o_ccount = o; o += al(utfx_dev::NCLS * 8);
  uint64_t o_small[utfx_dev::NCLS];
  for (int c = 0; c < utfx_dev::NCLS; ++c) {
    o_small[c] = o; o += al(ni * 4);
  }
  uint64_t o_plan[2], o_status[2], o_uitem[2], o_tiny[2];
  for (int d = 0; d < 2; ++d) {
    o_tiny[d] = o; o += al(ni * 4);
    o_plan[d] = o; o += al(plan_words * 8 * utfx_dev::STATUS_STRIDE);
    o_status[d] = o; o += al(nu * 8 * utfx_dev::STATUS_STRIDE);
    o_uitem[d] = o; o += al(nu * 4);
  }
  e = hipMalloc(&b.mem, o);
  if (e != hipSuccess) {
    b.mem = nullptr;
    b.cap_items = b.cap_units = 0;
    return e;
  }
  char* m = static_cast<char*>(b.mem);
  b.ws = reinterpret_cast<utfx_dev::WsHeader*>(m);
  b.unit_start = reinterpret_cast<unsigned long long*>(m + o_start);
  b.item_err = reinterpret_cast<unsigned long long*>(m + o_err);
  b.large = reinterpret_cast<uint32_t*>(m + o_large);
  b.cls_count = reinterpret_cast<unsigned long long*>(m + o_ccount);
  for (int c = 0; c < utfx_dev::NCLS; ++c) b.small[c] = reinterpret_cast<uint32_t*>(m + o_small[c]);
  for (int d = 0; d < 2; ++d) {
    b.tiny[d] = reinterpret_cast<uint32_t*>(m + o_tiny[d]);
    b.plan_status[d] = reinterpret_cast<unsigned long long*>(m + o_plan[d]);
    b.status[d] = reinterpret_cast<unsigned long long*>(m + o_status[d]);
    b.unit_item[d] = reinterpret_cast<uint32_t*>(m + o_uitem[d]);
  }
  b.cap_items = ni;
  b.cap_units = nu;
  return batch_ws_clear(b, s);
}

// Tunables of the batched call (utfx_set_batch_tuning).
struct BatchTuning {
  uint64_t small_max = utfx_dev::SMALL_MAX;  // largest string one wave walks
  uint32_t bs = 4;                           // tiles per large-item segment: 2 or 4
  uint32_t large_wgs = 2;                    // persistent large-segment workgroups per CU: 1 or 2
};

inline utfx_status batch_run(BatchWs& b, hipStream_t s, bool capturing, int num_cus, uint32_t dbg,
                             const BatchTuning& tun,
                             const uint8_t* in,
                             uint64_t in_bytes, uint8_t* out, uint64_t out_bytes, const utfx_item* d_items,
                             uint32_t n_items, uint64_t total_in_units, utfx_result* d_results, char* err,
                             size_t errlen) {
  using namespace utfx_dev;
  if (n_items == 0) return UTFX_OK;
  if ((!in && in_bytes) || (!out && out_bytes) || !d_items || !d_results) {
    snprintf(err, errlen, "null pointer");
    return UTFX_E_INVALID_ARG;
  }
  // segments of large items per direction: an item of n > small_max units has at most
  // n / seg + 2, and there are at most total / small_max such items
  const uint64_t seg_min = 8ull * BWG * tun.bs;  // the UTF-16 segment, in units, is the smaller
  const uint64_t cap_units = total_in_units / seg_min + 2 * (total_in_units / tun.small_max) + 2;
  if (capturing && (n_items > b.cap_items || cap_units > b.cap_units || b.launches >= (1ull << 24))) {
    snprintf(err, errlen, "batch workspace must grow during graph capture; make the same call once before capturing");
    return UTFX_E_INVALID_ARG;
  }
  hipError_t e = batch_ws_ensure(b, s, n_items, cap_units);
  if (e != hipSuccess) {
    snprintf(err, errlen, "batch workspace: %s", hipGetErrorString(e));
    return UTFX_E_DEVICE;
  }
  BatchArgs A;
  A.in = in;
  A.out = out;
  A.in_bytes = in_bytes;
  A.out_bytes = out_bytes;
  A.items = reinterpret_cast<const BItem*>(d_items);
  A.results = reinterpret_cast<Result*>(d_results);
  A.n_items = n_items;
  A.ws = b.ws;
  A.unit_start = b.unit_start;
  A.item_err = b.item_err;
  A.large = b.large;
  A.cls_count = b.cls_count;
  for (int c = 0; c < NCLS; ++c) A.small[c] = b.small[c];
  for (int d = 0; d < 2; ++d) {
    A.tiny[d] = b.tiny[d];
    A.status[d] = b.status[d];
    A.unit_item[d] = b.unit_item[d];
    A.plan_status[d] = b.plan_status[d];
  }
  A.cap_units = cap_units;
  A.total_in = total_in_units;
  // rows pay off on many strings; a call with few (a serving step) saves the launch
  A.rows = n_items >= TINY_ROWS_MIN;
  A.small_max = tun.small_max;
  A.bs = tun.bs;
  A.dbg = dbg;
  const uint32_t plan_blocks = (n_items + PLAN_WG * PLAN_ITEMS - 1) / (PLAN_WG * PLAN_ITEMS);
  // tiny waves: at most n/4 + 2 (four items per wave, per direction, rounded up)
  const uint32_t tiny_blocks = (uint32_t)((n_items / 4 + 2 + TINY_WG / 64 - 1) / (TINY_WG / 64));
  // the large segments: persistent grids of tun.large_wgs workgroups per CU (at most two
  // are resident: 128 VGPRs), fewer for a call with few segments; the wave-walked
  // items: one wave each
  const uint64_t cus = (uint64_t)(num_cus > 0 ? num_cus : 256);
  const uint64_t large_blocks = cap_units < tun.large_wgs * cus ? cap_units : tun.large_wgs * cus;
  const uint64_t small_blocks = (n_items + SMALL_WG / 64 - 1) / (SMALL_WG / 64);
  const uint32_t fin_blocks = n_items < 1024 ? n_items : 1024;
  hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, s, b.ws, b.cls_count);
  hipLaunchKernelGGL(k_batch_plan, dim3(plan_blocks), dim3(PLAN_WG), 0, s, A);
  if (A.rows) hipLaunchKernelGGL(k_batch_tiny, dim3(tiny_blocks), dim3(TINY_WG), 0, s, A);
  hipLaunchKernelGGL(k_batch_small, dim3((uint32_t)small_blocks), dim3(SMALL_WG), 0, s, A);
  if (tun.bs == 2) {
    hipLaunchKernelGGL((k_batch_large<0, 2>), dim3((uint32_t)large_blocks), dim3(BWG), 0, s, A);
    hipLaunchKernelGGL((k_batch_large<1, 2>), dim3((uint32_t)large_blocks), dim3(BWG), 0, s, A);
  } else {
    hipLaunchKernelGGL((k_batch_large<0, 4>), dim3((uint32_t)large_blocks), dim3(BWG), 0, s, A);
    hipLaunchKernelGGL((k_batch_large<1, 4>), dim3((uint32_t)large_blocks), dim3(BWG), 0, s, A);
  }
  hipLaunchKernelGGL(k_batch_fin, dim3(fin_blocks), dim3(FIN_WG), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(err, errlen, "batch launch: %s", hipGetErrorString(e));
    return UTFX_E_DEVICE;
  }
  b.launches++;
  return UTFX_OK;
}
