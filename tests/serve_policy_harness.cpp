// CPU harness for the server's packing and scheduling decisions (utfx_serve_policy.hpp):
// a mock executor on a virtual clock.  Requests arrive by a seeded Poisson process with a
// mix of sizes (some above the bulk threshold, some larger than an arena, some with a bad
// direction, some with pinned buffers); free slots take steps as the server does; a
// step's duration is a fixed cost plus its bytes over a bandwidth, with seeded jitter.
// Checked: every request completes exactly once or is rejected exactly when no slot can
// hold it; within a step, placements are 16-byte aligned, inside the arenas and disjoint
// (staged from the start, direct from the end); each queue is served in arrival order;
// steps hold 1..max_items requests; a bulk step starts only when no bulk step is in
// flight or no small request waits.  Some step launches fail (as a failed copy or
// batched call would): their requests must complete exactly once, through the failed
// list, with the slot free at once.  Prints "ok <counts>" or the first violation.
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <deque>
#include <random>
#include <vector>

#include "utfx_serve_policy.hpp"

using namespace utfx_srv;

struct MReq {
  uint64_t id, arrival, in_bytes, out_bytes;
  uint32_t dir;
  bool pinned_in, pinned_out, bulk;
};

struct MSlot {
  bool busy = false, bulk = false;
  uint64_t end = 0;
  std::vector<uint64_t> ids;
};

static int fail(const char* what, uint64_t a, uint64_t b) {
  printf("FAIL %s %llu %llu\n", what, (unsigned long long)a, (unsigned long long)b);
  return 1;
}

static int run(uint64_t seed, uint32_t n_slots, uint32_t max_items, double rate_per_us) {
  const uint64_t kBulk = 1 << 20, kArenaIn = 8 << 20, kArenaOut = 24 << 20, kDirect = 64 << 10;
  std::mt19937_64 g(seed);
  std::exponential_distribution<double> gap(rate_per_us);
  std::lognormal_distribution<double> size(8.0, 2.0);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const uint32_t n = 20000;
  std::vector<MReq> reqs(n);
  double t = 0;
  for (uint32_t i = 0; i < n; ++i) {
    t += gap(g);
    MReq& r = reqs[i];
    r.id = i;
    r.arrival = (uint64_t)t;
    uint64_t len = std::min<uint64_t>((uint64_t)size(g) + 1, 40ull << 20);
    if (u(g) < 0.01) len = (uint64_t)(u(g) * (kArenaIn / 2)) + kBulk;  // bulk
    r.dir = u(g) < 0.003 ? 2 : (u(g) < 0.5 ? 0 : 1);
    r.in_bytes = r.dir == 1 ? 2 * (len / 2 + 1) : len;
    r.out_bytes = r.dir == 1 ? 3 * (r.in_bytes / 2) : 2 * r.in_bytes;
    r.pinned_in = u(g) < 0.3;
    r.pinned_out = u(g) < 0.3;
    r.bulk = r.in_bytes >= kBulk;
  }
  const PackLimits lim{kArenaIn, kArenaOut, max_items, kDirect};
  std::vector<MSlot> slots(n_slots);
  std::deque<uint64_t> small, bulk;
  std::vector<int> done(n, 0);
  std::vector<int> rejected(n, 0);
  std::vector<int> failed_ids(n, 0);
  FailedRequests failed;
  uint64_t last_small = 0, last_bulk = 0, now = 0, steps = 0, n_done = 0, n_rej = 0, n_fail = 0, failed_steps = 0;
  bool seen_small = false, seen_bulk = false;
  uint32_t next = 0;
  while (n_done + n_rej < n) {
    // failed steps' requests complete first (the server reports them on its next call)
    while (!failed.empty()) {
      const uint64_t id = failed.pop();
      if (done[id]++) return fail("completed twice", id, 0);
      if (!failed_ids[id]) return fail("completed as failed without a failed step", id, 0);
      ++n_done;
      ++n_fail;
    }
    if (n_done + n_rej >= n) break;
    // the next event: an arrival or a step's end
    uint64_t te = UINT64_MAX;
    if (next < n) te = reqs[next].arrival;
    for (auto& s : slots)
      if (s.busy) te = std::min(te, s.end);
    if (te == UINT64_MAX) return fail("stuck: requests wait but nothing is scheduled", n_done, n_rej);
    now = std::max(now, te);
    while (next < n && reqs[next].arrival <= now) {
      (reqs[next].bulk ? bulk : small).push_back(next);
      ++next;
    }
    for (auto& s : slots) {
      if (!s.busy || s.end > now) continue;
      for (uint64_t id : s.ids) {
        if (done[id]++) return fail("completed twice", id, 0);
        ++n_done;
      }
      s.busy = false;
      s.ids.clear();
    }
    bool bulk_busy = false;
    for (auto& s : slots) bulk_busy |= s.busy && s.bulk;
    for (auto& s : slots) {
      if (s.busy) continue;
      const int which = pick_queue(!bulk.empty(), !small.empty(), bulk_busy);
      if (which < 0) continue;
      if (which == 1 && bulk_busy && !small.empty()) return fail("bulk step while small requests wait", now, 0);
      std::deque<uint64_t>& q = which == 1 ? bulk : small;
      StepPacker pk(lim);
      struct Iv { uint64_t lo, hi; };
      std::vector<Iv> ins, outs;
      uint64_t bytes = 0;
      while (!q.empty()) {
        const MReq& r = reqs[q.front()];
        Placement p;
        const PackVerdict v = pk.place(ReqShape{r.in_bytes, r.out_bytes, r.dir, r.pinned_in, r.pinned_out}, &p);
        if (v == PACK_REJECT) {
          const bool fits = r.dir <= 1 && r.in_bytes <= kArenaIn && r.out_bytes <= kArenaOut;
          if (fits) return fail("rejected a request a slot can hold", r.id, r.in_bytes);
          if (rejected[r.id]++) return fail("rejected twice", r.id, 0);
          ++n_rej;
          q.pop_front();
          continue;
        }
        if (v == PACK_FULL) {
          if (s.ids.empty()) return fail("an empty step is full", r.id, r.in_bytes);
          break;
        }
        if ((p.in_off | p.out_off) & 15) return fail("unaligned placement", r.id, p.in_off);
        if (p.in_off + r.in_bytes > kArenaIn || p.out_off + r.out_bytes > kArenaOut)
          return fail("placement outside the arena", r.id, p.in_off);
        if (p.direct_in != (r.pinned_in && r.in_bytes >= kDirect) ||
            p.direct_out != (r.pinned_out && r.out_bytes >= kDirect))
          return fail("wrong copy route", r.id, 0);
        ins.push_back({p.in_off, p.in_off + r.in_bytes});
        outs.push_back({p.out_off, p.out_off + r.out_bytes});
        uint64_t& last = which == 1 ? last_bulk : last_small;
        bool& seen = which == 1 ? seen_bulk : seen_small;
        if (seen && r.id <= last) return fail("queue served out of order", r.id, last);
        seen = true;
        last = r.id;
        s.ids.push_back(r.id);
        bytes += r.in_bytes + r.out_bytes;
        q.pop_front();
      }
      if (s.ids.size() > max_items) return fail("step too large", s.ids.size(), max_items);
      for (auto* v : {&ins, &outs}) {
        std::sort(v->begin(), v->end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
        for (size_t k = 1; k < v->size(); ++k)
          if ((*v)[k].lo < (*v)[k - 1].hi) return fail("overlapping placements", (*v)[k].lo, (*v)[k - 1].hi);
      }
      if (s.ids.empty()) continue;
      if (u(g) < 0.02) {  // the launch fails: the slot stays free, its requests fail once
        for (uint64_t id : s.ids) {
          if (failed_ids[id]++) return fail("failed twice", id, 0);
          failed.add(id);
        }
        s.ids.clear();
        ++failed_steps;
        continue;
      }
      s.busy = true;
      s.bulk = which == 1;
      bulk_busy |= s.bulk;
      s.end = now + 20 + bytes / 2000 + (uint64_t)(u(g) * 30);  // us: launch cost + bytes at ~2 GB/s + jitter
      ++steps;
    }
  }
  for (uint32_t i = 0; i < n; ++i)
    if (done[i] + rejected[i] != 1) return fail("request lost", i, 0);
  if (failed_steps == 0 || n_fail == 0) return fail("no failed step was exercised", failed_steps, n_fail);
  printf("ok seed=%llu slots=%u max_items=%u steps=%llu done=%llu rejected=%llu failed_steps=%llu failed=%llu\n",
         (unsigned long long)seed, n_slots, max_items, (unsigned long long)steps, (unsigned long long)n_done,
         (unsigned long long)n_rej, (unsigned long long)failed_steps, (unsigned long long)n_fail);
  return 0;
}

int main() {
  int rc = 0;
  rc |= run(1, 1, 65536, 0.05);
  rc |= run(2, 2, 64, 0.2);
  rc |= run(3, 3, 4096, 1.0);
  rc |= run(4, 4, 8, 0.5);
  return rc;
}
