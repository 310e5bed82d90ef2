// The server's decisions, free of HIP: where a request goes in a step's arenas, when a
// step is full, which requests are rejected, and which queue a free slot serves.  The
// server (utfx_serve.hpp) calls these; a CPU harness with a mock executor on a virtual
// clock tests them without a GPU.
#pragma once

#include <stdint.h>

#include <deque>

namespace utfx_srv {

// What the policy needs to know of a request.
struct ReqShape {
  uint64_t in_bytes;
  uint64_t out_bytes;
  uint32_t dir;     // 0 = UTF-8 -> UTF-16LE, 1 = UTF-16LE -> UTF-8; anything else is rejected
  bool pinned_in;   // the caller's input buffer is pinned host memory
  bool pinned_out;  // the caller's output buffer is pinned host memory
  bool device = false;  // payload and output live in device memory (never staged)
};

struct PackLimits {
  uint64_t arena_in;    // bytes of a slot's input arena
  uint64_t arena_out;   // bytes of a slot's output arena
  uint32_t max_items;   // requests per step
  uint64_t direct_min;  // pinned buffers of at least this many bytes are copied directly
};

// Where a placed request lives in the step's arenas.  Staged data (copied through the
// slot's pinned mirror) grows from the start of each arena, 16-byte aligned; direct data
// (copied straight from or to the caller's pinned buffer, or by the gather and scatter
// kernels for device-resident requests) grows down from the end.
struct Placement {
  uint64_t in_off;
  uint64_t out_off;
  bool direct_in;
  bool direct_out;
};

enum PackVerdict { PACK_PLACED, PACK_REJECT, PACK_FULL };

inline uint64_t al16(uint64_t x) { return (x + 15) & ~15ull; }

// Packs one step, request by request in queue order.  REJECT: no slot can ever hold the
// request (bad direction, or larger than an arena); FULL: it does not fit in what is left
// of this step (the step is launched and the request waits for the next one).
struct StepPacker {
  PackLimits lim;
  uint64_t in_lo = 0, out_lo = 0, in_hi, out_hi;
  uint32_t count = 0;

  explicit StepPacker(const PackLimits& l) : lim(l), in_hi(l.arena_in), out_hi(l.arena_out) {}

  PackVerdict place(const ReqShape& r, Placement* p) {
    if (r.dir > 1 || r.in_bytes > lim.arena_in || r.out_bytes > lim.arena_out) return PACK_REJECT;
    if (count >= lim.max_items) return PACK_FULL;
    const bool din = r.device || (r.in_bytes >= lim.direct_min && r.pinned_in);
    const bool dout = r.device || (r.out_bytes >= lim.direct_min && r.pinned_out);
    uint64_t io, oo, nlo = in_lo, nhi = in_hi, olo = out_lo, ohi = out_hi;
    if (din) {
      if (r.in_bytes > nhi) return PACK_FULL;
      io = nhi = (nhi - r.in_bytes) & ~15ull;
    } else {
      io = al16(nlo);
      nlo = io + r.in_bytes;
    }
    if (dout) {
      if (r.out_bytes > ohi) return PACK_FULL;
      oo = ohi = (ohi - r.out_bytes) & ~15ull;
    } else {
      oo = al16(olo);
      olo = oo + r.out_bytes;
    }
    if (nlo > nhi || olo > ohi) return PACK_FULL;
    in_lo = nlo;
    in_hi = nhi;
    out_lo = olo;
    out_hi = ohi;
    ++count;
    p->in_off = io;
    p->out_off = oo;
    p->direct_in = din;
    p->direct_out = dout;
    return PACK_PLACED;
  }

  uint64_t staged_in_bytes() const { return in_lo; }    // bytes of the input mirror to copy
  uint64_t staged_out_bytes() const { return out_lo; }  // bytes of the output mirror to copy back
};

// Requests of steps that could not be launched (a copy or the batched call failed to
// queue).  The slot is free again at once; each of its requests completes exactly once,
// with a device error, on a later progress call (never with the results of an earlier
// step left in the slot's buffers).
struct FailedRequests {
  std::deque<uint64_t> tags;
  void add(uint64_t tag) { tags.push_back(tag); }
  bool empty() const { return tags.empty(); }
  uint64_t pop() {
    const uint64_t t = tags.front();
    tags.pop_front();
    return t;
  }
};

// Which queue a free slot serves: 1 = bulk, 0 = small, -1 = none.  A bulk step is
// launched when none is in flight, and more bulk steps only while no small request waits,
// so small requests are never stuck behind several large ones.
inline int pick_queue(bool bulk_waiting, bool small_waiting, bool bulk_in_flight) {
  if (bulk_waiting && (!bulk_in_flight || !small_waiting)) return 1;
  if (small_waiting) return 0;
  return -1;
}

}  // namespace utfx_srv
