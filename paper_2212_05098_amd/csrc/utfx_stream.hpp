// Streams: the cut between two chunks.
//
// A stream call transcodes the carried units of the previous call followed by the new
// chunk, except for a character left unfinished at the chunk's end, which it carries on.
// The input therefore advances by whole sequences only (section 6), and a high surrogate
// ending a chunk is paired with the next chunk's first word (the surrogate carry c of
// section 7.4).  The work of a call is split in two:
//
//   piece 1: the carried units followed by the first h units of the chunk, the one
//            character across the cut, staged and transcoded by k_stream_edge with
//            the batched path's one-wave transcoder;
//   piece 2: chunk[h, n), an ordinary single-buffer transcode in place, its output
//            placed after piece 1's.
//
// h and piece 1's output length are known to the host before the launches: the
// previous call's k_stream_edge recorded, for the character it carried, how many units
// it still needs and how many output units it makes if valid.  Piece 2 runs to the end
// of the chunk; when the chunk ends in an unfinished character starting at t, piece 2
// reports its (truncation) error exactly at t, with the output of chunk[h, t) complete,
// and the host turns that into success with chunk[t, n) carried.  The staged character
// is judged by the same kernels as everything else, so it gets the verdict it has in the
// concatenated input: piece 1 holds all of its units (or, at the end of the stream, all
// there are), and the verdict on a character depends only on its own units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "utfx_batch.hpp"
#include "utfx_device.hpp"

namespace utfx_dev {

struct StreamEdge {
  uint64_t t;         // the unfinished character at the chunk's end starts at t (t = n: none)
  uint32_t n_keep;    // units carried to the next call
  uint32_t keep_need; // units the carried character still needs
  uint32_t keep_out;  // output units of the carried character once complete and valid
  uint32_t pad;
  uint8_t keep[8];    // the carried units as they are in memory
};

// Device memory of a stream call: piece 1 staged, transcoded and copied out from here.
struct StreamDev {
  Result r1;          // piece 1's result before the caller's capacity is applied
  uint8_t stage[16];  // piece 1 (UTF-16 staged little-endian)
  uint8_t out1[16];   // piece 1's output before it is copied out (UTF-16 little-endian)
};

// What the host reads after the call's one synchronisation; pinned host memory that the
// kernels write through its device address.
struct StreamRec {
  Result r[2];        // results of piece 1 and piece 2
  StreamEdge e;
};

enum : uint32_t { SE_IN16 = 1u, SE_BE = 2u, SE_FINAL = 4u };

// Length in bytes of the character that a lead byte (C0..FF) starts (Table 1); bytes
// that are not allowed as leads get a length too, and their error is found when the
// character is transcoded.
__device__ __forceinline__ uint32_t se_len_of_lead(uint32_t b) { return b >= 0xF0u ? 4u : b >= 0xE0u ? 3u : 2u; }

// One wave.  Lane 0 looks at the units next to the two cuts: it stages piece 1 (the nc
// carried units, packed little-endian in `carry`, then chunk[0, h)) and finds the
// unfinished character at the chunk's end (not before h).  With grow != 0 the chunk
// does not finish the carried character (h = n) and is carried along with it instead.
// Then the wave transcodes piece 1 into out1 and lane 0 copies it to out[0, cap) and
// writes its result to rec->r[0]; the cut goes to rec->e.
__global__ void __launch_bounds__(64) k_stream_edge(StreamDev* d, StreamRec* rec, const void* in_v, uint64_t n,
                                                    uint64_t h, uint32_t carry, uint32_t nc, uint32_t flags,
                                                    uint32_t grow, void* out, uint64_t cap) {
  __shared__ __attribute__((aligned(16))) uint8_t wstage[WSTAGE];
  const uint32_t lane = threadIdx.x;
  const bool fin = (flags & SE_FINAL) != 0;
  const bool in16 = (flags & SE_IN16) != 0, be = (flags & SE_BE) != 0;
  const bool piece1 = nc > 0 && !grow;
  if (lane == 0) {
    uint32_t keep[2] = {0u, 0u};
    uint32_t stage[2] = {0u, 0u};
    auto put = [](uint32_t* a, uint32_t i, uint32_t byte) { a[i >> 2] |= (byte & 0xFFu) << (8u * (i & 3u)); };
    uint64_t t = n;
    uint32_t n_keep = 0, need = 0, outu = 0;

    if (!(flags & SE_IN16)) {
      const uint8_t* in = static_cast<const uint8_t*>(in_v);
      for (uint32_t i = 0; i < nc; ++i) put(stage, i, carry >> (8u * i));
      for (uint32_t i = 0; i < h; ++i) put(stage, nc + i, in[i]);
      if (grow) {
        for (uint32_t i = 0; i < nc + h; ++i) put(keep, i, i < nc ? carry >> (8u * i) : in[i - nc]);
        n_keep = nc + static_cast<uint32_t>(h);
        uint32_t lead = carry & 0xFFu;
        need = se_len_of_lead(lead) - n_keep;
        outu = lead >= 0xF0u ? 2u : 1u;
      } else {
        if (!fin) {
          for (uint64_t k = 1; k <= 3 && k <= n - h; ++k) {
            uint32_t b = in[n - k];
            if (b < 0x80u) break;  // ASCII ends the chunk: nothing unfinished
            if (b >= 0xC0u) {      // the last lead byte: unfinished if it wants more
              uint32_t len = se_len_of_lead(b);
              if (len > k) {
                t = n - k;
                need = len - static_cast<uint32_t>(k);
                outu = b >= 0xF0u ? 2u : 1u;  // one UTF-16 word, two for a 4-byte character
              }
              break;
            }
          }
        }
        n_keep = static_cast<uint32_t>(n - t);
        for (uint32_t i = 0; i < n_keep; ++i) put(keep, i, in[t + i]);
      }
    } else {
      const uint16_t* in = static_cast<const uint16_t*>(in_v);
      if (nc) {  // staged in little-endian order
        uint32_t w = carry & 0xFFFFu;
        if (be) w = bswap16(w);
        put(stage, 0, w);
        put(stage, 1, w >> 8);
      }
      if (h) {
        uint32_t w = in[0];
        if (be) w = bswap16(w);
        put(stage, 2 * nc, w);
        put(stage, 2 * nc + 1, w >> 8);
      }
      if (grow) {  // an empty chunk: the high surrogate stays carried
        put(keep, 0, carry);
        put(keep, 1, carry >> 8);
        n_keep = 1;
        need = 1;
        outu = 4;
      } else if (!fin && n > h) {
        uint32_t w = in[n - 1];
        if ((((be ? bswap16(w) : w)) & 0xFC00u) == 0xD800u) {  // a high surrogate waits for its pair
          t = n - 1;
          n_keep = 1;
          need = 1;
          outu = 4;  // a supplementary character: four UTF-8 bytes
          put(keep, 0, w);
          put(keep, 1, w >> 8);
        }
      }
    }
    StreamEdge e;
    e.t = t;
    e.n_keep = n_keep;
    e.keep_need = need;
    e.keep_out = outu;
    e.pad = 0;
    uint32_t* ek = reinterpret_cast<uint32_t*>(e.keep);
    ek[0] = keep[0];
    ek[1] = keep[1];
    rec->e = e;
    uint32_t* ds = reinterpret_cast<uint32_t*>(d->stage);
    ds[0] = stage[0];
    ds[1] = stage[1];
  }  // lane 0
  if (!piece1) return;  // wave-uniform
  __threadfence();
  __syncthreads();
  // piece 1 through the one-wave transcoder, into out1 (room for anything four input
  // units can make)
  const uintptr_t alo = reinterpret_cast<uintptr_t>(d->stage), ahi = alo + sizeof(d->stage);
  const uint64_t n1 = nc + h;
  if (!in16)
    wave_u8_to_u16(d->stage, n1, reinterpret_cast<uint16_t*>(d->out1), sizeof(d->out1) / 2,
                   reinterpret_cast<uint16_t*>(wstage), &d->r1, alo, ahi);
  else
    wave_u16_to_u8(reinterpret_cast<const uint16_t*>(d->stage), n1, d->out1, sizeof(d->out1), wstage, &d->r1,
                   alo, ahi);
  __threadfence();
  __syncthreads();
  if (lane != 0) return;
  Result r = d->r1;
  uint64_t w = r.status == ST_OUTPUT_TOO_SMALL ? 0 : r.written;
  if (r.status == ST_OK && r.count > cap) {
    r.status = ST_OUTPUT_TOO_SMALL;
    r.written = 0;
    w = 0;
  }
  if (w > cap) w = cap;
  if (!in16) {
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(d->out1);
    uint16_t* o16 = static_cast<uint16_t*>(out);
    for (uint64_t i = 0; i < w; ++i) o16[i] = static_cast<uint16_t>(be ? bswap16(s16[i]) : s16[i]);
  } else {
    uint8_t* o8 = static_cast<uint8_t*>(out);
    for (uint64_t i = 0; i < w; ++i) o8[i] = d->out1[i];
  }
  write_result(&rec->r[0], r.status, r.count, r.written);
}

}  // namespace utfx_dev
