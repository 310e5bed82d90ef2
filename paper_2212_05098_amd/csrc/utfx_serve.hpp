// utfx_serve.hpp -- continuous-batching server over the batched call (host code).
//
// Requests (host payloads) queue up; whenever one of the server's in-flight slots is
// free, one step takes every queued request that fits the slot's arenas (admission by
// free arena bytes and item slots), packs the payloads into the slot's pinned staging
// buffer, and on the slot's own stream copies them to the device, runs one batched
// call, and copies results and outputs back.  Requests that arrive while steps run
// join the next step (continuous batching); with two or more slots a step is packed
// and launched while earlier ones are still on the GPU.  Requests of kBulkMin input
// bytes or more queue apart and go to bulk steps, one in flight while small requests
// wait, so that the many small requests never wait behind a multi-MiB transfer.  Completion copies each
// request's output to its destination and reports its result.  Single-threaded: the
// caller drives it with utfx_server_progress, or replays a whole arrival trace in real
// time with utfx_server_replay.  Device-resident requests (payload and output in device
// memory) are gathered into the arena and scattered back by two kernels per step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <time.h>

#include <deque>
#include <new>
#include <vector>

#include "utfx.h"
#include "utfx_serve_policy.hpp"

namespace utfx_srv {

struct Req {
  uint64_t tag;
  const uint8_t* data;
  uint64_t len;       // input units
  uint32_t dir;
  uint8_t* out;
  uint64_t out_cap;   // output units
  bool dev;           // data and out are device addresses
};

// One piece (at most kPiece bytes) of a device-resident request's payload or output:
// its device address, its place in the step's arena (16-byte aligned), its size, and
// for outputs the item, the output unit size and the piece's offset in the output.
constexpr uint64_t kPiece = 16 << 10;
struct DevCopy {
  uint64_t ptr;
  uint64_t off;
  uint64_t bytes;     // gather: payload bytes of the piece; scatter: its capacity in bytes
  uint64_t start;     // scatter: byte offset of the piece in the request's output
  uint32_t item;
  uint32_t unit;      // scatter: output bytes per unit
};

// Bytes [a, a + 16) of the 32 bytes lo:hi (a in 0..15, wave-uniform).
__device__ __forceinline__ uint4 funnel16(const uint4 lo, const uint4 hi, uint32_t a) {
  const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  const uint32_t r = a & 3;
  uint4 o;
  switch (a >> 2) {
    case 0: o = {__builtin_amdgcn_alignbyte(w[1], w[0], r), __builtin_amdgcn_alignbyte(w[2], w[1], r),
                 __builtin_amdgcn_alignbyte(w[3], w[2], r), __builtin_amdgcn_alignbyte(w[4], w[3], r)}; break;
    case 1: o = {__builtin_amdgcn_alignbyte(w[2], w[1], r), __builtin_amdgcn_alignbyte(w[3], w[2], r),
                 __builtin_amdgcn_alignbyte(w[4], w[3], r), __builtin_amdgcn_alignbyte(w[5], w[4], r)}; break;
    case 2: o = {__builtin_amdgcn_alignbyte(w[3], w[2], r), __builtin_amdgcn_alignbyte(w[4], w[3], r),
                 __builtin_amdgcn_alignbyte(w[5], w[4], r), __builtin_amdgcn_alignbyte(w[6], w[5], r)}; break;
    default: o = {__builtin_amdgcn_alignbyte(w[4], w[3], r), __builtin_amdgcn_alignbyte(w[5], w[4], r),
                  __builtin_amdgcn_alignbyte(w[6], w[5], r), __builtin_amdgcn_alignbyte(w[7], w[6], r)}; break;
  }
  return o;
}

__device__ __forceinline__ void store_bytes(uint8_t* p, const uint4 v, uint32_t i0, uint32_t i1) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  for (uint32_t i = i0; i < i1; ++i) p[i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
}

// Gathers device-resident payload pieces into the step's input arena, one workgroup per
// piece (grid-strided), 16 bytes per thread: the source (any alignment) is read as the
// aligned 16-byte blocks that hold the chunk's bytes (a block holding at least one byte
// of the buffer never crosses a page) and funnel-shifted; the arena side is aligned.
__global__ void __launch_bounds__(256) k_srv_gather(const DevCopy* c, uint32_t n, uint8_t* arena) {
  for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
    const DevCopy d = c[k];
    const uint32_t a = (uint32_t)(d.ptr & 15);
    const uint8_t* b0 = reinterpret_cast<const uint8_t*>(d.ptr - a);
    uint8_t* dst = arena + d.off;
    const uint64_t nch = (d.bytes + 15) / 16;
    for (uint64_t ch = threadIdx.x; ch < nch; ch += blockDim.x) {
      const uint4 lo = *reinterpret_cast<const uint4*>(b0 + 16 * ch);
      uint4 v = lo;
      if (a) {
        uint4 hi = {0, 0, 0, 0};
        if (16 * ch + 16 - a < d.bytes) hi = *reinterpret_cast<const uint4*>(b0 + 16 * ch + 16);
        v = funnel16(lo, hi, a);
      }
      if (16 * ch + 16 <= d.bytes) *reinterpret_cast<uint4*>(dst + 16 * ch) = v;
      else store_bytes(dst + 16 * ch, v, 0, (uint32_t)(d.bytes - 16 * ch));
    }
  }
}

// Copies the valid prefix of each device-resident request's output (written units, at
// most its capacity; nothing on OUTPUT_TOO_SMALL) from the output arena to its buffer,
// piece by piece: whole aligned 16-byte blocks of the destination are stored at once,
// the partly covered first and last blocks byte by byte, so nothing outside the
// prefix is touched.
__global__ void __launch_bounds__(256) k_srv_scatter(const DevCopy* c, uint32_t n, const uint8_t* arena,
                                                     const utfx_result* res) {
  for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
    const DevCopy d = c[k];
    const utfx_result r = res[d.item];
    if (r.status == UTFX_E_OUTPUT_TOO_SMALL) continue;
    const uint64_t total = r.written * d.unit;
    if (total <= d.start) continue;
    const uint64_t nb = total - d.start < d.bytes ? total - d.start : d.bytes;
    const uint8_t* src = arena + d.off;
    const uint32_t a = (uint32_t)(d.ptr & 15);
    uint8_t* B0 = reinterpret_cast<uint8_t*>(d.ptr - a);
    const uint64_t nblk = (a + nb + 15) / 16;
    for (uint64_t j = threadIdx.x; j < nblk; j += blockDim.x) {
      // destination block j holds output bytes [16j - a, 16j - a + 16)
      uint4 v;
      if (a == 0) {
        v = *reinterpret_cast<const uint4*>(src + 16 * j);
      } else {
        uint4 lo = {0, 0, 0, 0}, hi = {0, 0, 0, 0};
        if (j >= 1) lo = *reinterpret_cast<const uint4*>(src + 16 * (j - 1));
        if (16 * j < nb) hi = *reinterpret_cast<const uint4*>(src + 16 * j);
        v = funnel16(lo, hi, 16 - a);
      }
      const int64_t s0 = (int64_t)(16 * j) - (int64_t)a;
      if (s0 >= 0 && (uint64_t)s0 + 16 <= nb) {
        *reinterpret_cast<uint4*>(B0 + 16 * j) = v;
      } else {
        const uint32_t i0 = s0 < 0 ? (uint32_t)(-s0) : 0u;
        const uint32_t i1 = (uint64_t)(s0 + 16) > nb ? (uint32_t)((int64_t)nb - s0) : 16u;
        store_bytes(B0 + 16 * j, v, i0, i1);
      }
    }
  }
}

struct Slot {
  utfx_ctx* ctx = nullptr;  // own context: batch workspaces are per context
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* h_in = nullptr;
  uint8_t* d_in = nullptr;
  uint8_t* h_out = nullptr;
  uint8_t* d_out = nullptr;
  utfx_item* h_items = nullptr;
  utfx_item* d_items = nullptr;
  utfx_result* h_res = nullptr;
  utfx_result* d_res = nullptr;
  DevCopy* h_gather = nullptr;      // device-resident requests of the step (pinned)
  DevCopy* d_gather = nullptr;
  DevCopy* h_scatter = nullptr;
  DevCopy* d_scatter = nullptr;
  std::vector<Req> reqs;
  std::vector<uint8_t> direct_out;  // per request: output copied straight to its buffer
  std::vector<uint64_t> direct_in_off, direct_out_off;
  bool busy = false;
  bool bulk = false;  // the step in flight holds bulk requests
};

// Requests at least this large whose host buffers are pinned skip the staging copy:
// their payload and output move by DMA straight between the request's buffer and the
// device arena.
constexpr uint64_t kDirectMin = 64 << 10;

// Requests at least this large (input bytes) are bulk requests.
constexpr uint64_t kBulkMin = 1 << 20;

inline bool is_pinned(const void* p) {
  hipPointerAttribute_t a;
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // pageable memory: clear the error the query left
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

inline uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

}  // namespace utfx_srv

struct utfx_server {
  utfx_server_config cfg;
  std::deque<utfx_srv::Req> pending;       // small requests, arrival order
  std::deque<utfx_srv::Req> pending_bulk;  // bulk requests, arrival order
  std::deque<uint64_t> rejected;  // tags of requests no slot can ever hold
  utfx_srv::FailedRequests failed;  // tags of requests whose step could not be launched
  std::vector<utfx_srv::Slot> slots;
  uint64_t steps = 0;
  uint64_t items_total = 0;
  char err[256];
};

namespace utfx_srv {

inline void free_slot(Slot& s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  if (s.ctx) utfx_destroy(s.ctx);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.h_in) (void)hipHostFree(s.h_in);
  if (s.h_out) (void)hipHostFree(s.h_out);
  if (s.h_items) (void)hipHostFree(s.h_items);
  if (s.h_res) (void)hipHostFree(s.h_res);
  if (s.d_in) (void)hipFree(s.d_in);
  if (s.d_out) (void)hipFree(s.d_out);
  if (s.d_items) (void)hipFree(s.d_items);
  if (s.d_res) (void)hipFree(s.d_res);
  if (s.h_gather) (void)hipHostFree(s.h_gather);
  if (s.d_gather) (void)hipFree(s.d_gather);
  s = Slot();
}

inline uint64_t gather_cap(const utfx_server_config& c) { return c.max_items + c.arena_in_bytes / kPiece + 1; }
inline uint64_t scatter_cap(const utfx_server_config& c) { return c.max_items + c.arena_out_bytes / kPiece + 1; }

inline hipError_t alloc_slot(Slot& s, const utfx_server_config& c) {
  hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_in, c.arena_in_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_out, c.arena_out_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_items, c.max_items * sizeof(utfx_item), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_res, c.max_items * sizeof(utfx_result), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_in, c.arena_in_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_out, c.arena_out_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_items, c.max_items * sizeof(utfx_item));
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_res, c.max_items * sizeof(utfx_result));
  // gather list, then scatter list, in one allocation each side: a request takes one
  // piece per kPiece bytes (or part), so a step has at most max_items + arena / kPiece
  const uint64_t ng = gather_cap(c), ns = scatter_cap(c);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_gather, (ng + ns) * sizeof(DevCopy), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_gather, (ng + ns) * sizeof(DevCopy));
  if (e == hipSuccess) {
    s.h_scatter = s.h_gather + ng;
    s.d_scatter = s.d_gather + ng;
  }
  if (e == hipSuccess && utfx_create(&s.ctx, s.stream) != UTFX_OK) e = hipErrorOutOfMemory;
  return e;
}

// Host<->device copies of every size class a step issues, on the slot's stream.
inline hipError_t warm_copies(Slot& s, const utfx_server_config& c) {
  const uint64_t sizes[] = {64, 4096, 64 << 10, 1 << 20, 16 << 20, 1ull << 62};
  hipError_t e = hipSuccess;
  for (uint64_t z : sizes) {
    const uint64_t zi = z < c.arena_in_bytes ? z : c.arena_in_bytes;
    const uint64_t zo = z < c.arena_out_bytes ? z : c.arena_out_bytes;
    if (e == hipSuccess) e = hipMemcpyAsync(s.d_in, s.h_in, zi, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_out, s.d_out, zo, hipMemcpyDeviceToHost, s.stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.h_res, s.d_res, c.max_items * sizeof(utfx_result), hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.d_items, s.h_items, c.max_items * sizeof(utfx_item), hipMemcpyHostToDevice, s.stream);
  return e;
}

// Bytes a request needs in the input and output arenas.
inline uint64_t in_bytes(const Req& r) { return r.len * (r.dir ? 2 : 1); }
inline uint64_t out_bytes(const Req& r) { return r.out_cap * (r.dir ? 1 : 2); }

// Packs every request of queue q that fits into slot s and launches the step.  Returns
// the number of requests taken.  A request no slot can hold is rejected (it completes
// with UTFX_E_INVALID_ARG on the next progress call).  If the step cannot be launched,
// its requests complete with UTFX_E_DEVICE and the slot stays free.
inline uint32_t launch_step(utfx_server* S, Slot& s, std::deque<Req>& q, bool bulk) {
  const utfx_server_config& c = S->cfg;
  StepPacker pk(PackLimits{c.arena_in_bytes, c.arena_out_bytes, c.max_items, kDirectMin});
  uint64_t units = 0;
  s.reqs.clear();
  s.direct_out.clear();
  s.direct_in_off.clear();
  s.direct_out_off.clear();
  std::vector<uint32_t> direct_in_idx;
  uint32_t n_gather = 0, n_scatter = 0;
  while (!q.empty()) {
    const Req& r = q.front();
    ReqShape sh{in_bytes(r), out_bytes(r), r.dir, !r.dev && in_bytes(r) >= kDirectMin && is_pinned(r.data),
                !r.dev && out_bytes(r) >= kDirectMin && is_pinned(r.out)};
    sh.device = r.dev;
    Placement pl;
    const PackVerdict v = pk.place(sh, &pl);
    if (v == PACK_REJECT) {
      S->rejected.push_back(r.tag);
      q.pop_front();
      continue;
    }
    if (v == PACK_FULL) break;  // no room left in this step
    const uint64_t io = pl.in_off, oo = pl.out_off;
    const bool din = pl.direct_in, dout = pl.direct_out;
    if (r.dev) {
      const uint32_t item = (uint32_t)s.reqs.size();
      for (uint64_t p0 = 0; p0 < in_bytes(r); p0 += kPiece) {
        const uint64_t nb = in_bytes(r) - p0 < kPiece ? in_bytes(r) - p0 : kPiece;
        s.h_gather[n_gather++] = DevCopy{(uint64_t)(uintptr_t)r.data + p0, io + p0, nb, 0, item, 0};
      }
      for (uint64_t p0 = 0; p0 < out_bytes(r); p0 += kPiece) {
        const uint64_t nb = out_bytes(r) - p0 < kPiece ? out_bytes(r) - p0 : kPiece;
        s.h_scatter[n_scatter++] = DevCopy{(uint64_t)(uintptr_t)r.out + p0, oo + p0, nb, p0, item, r.dir ? 1u : 2u};
      }
    } else if (din) {
      direct_in_idx.push_back((uint32_t)s.reqs.size());
    } else if (in_bytes(r)) {
      memcpy(s.h_in + io, r.data, in_bytes(r));
    }
    utfx_item& it = s.h_items[s.reqs.size()];
    it.in_off = io;
    it.in_len = r.len;
    it.out_off = oo;
    it.out_cap = r.out_cap;
    it.dir = r.dir;
    it.pad = 0;
    units += r.len;
    s.reqs.push_back(r);
    s.direct_out.push_back(dout ? 1 : 0);
    q.pop_front();
  }
  const uint32_t n = (uint32_t)s.reqs.size();
  if (!n) return 0;
  hipError_t e = hipMemcpyAsync(s.d_items, s.h_items, n * sizeof(utfx_item), hipMemcpyHostToDevice, s.stream);
  const uint64_t in_lo = pk.staged_in_bytes(), out_lo = pk.staged_out_bytes();
  if (e == hipSuccess && in_lo) e = hipMemcpyAsync(s.d_in, s.h_in, in_lo, hipMemcpyHostToDevice, s.stream);
  for (uint32_t k : direct_in_idx) {
    if (e != hipSuccess) break;
    e = hipMemcpyAsync(s.d_in + s.h_items[k].in_off, s.reqs[k].data, in_bytes(s.reqs[k]), hipMemcpyHostToDevice,
                       s.stream);
  }
  if (e == hipSuccess && n_gather)
    e = hipMemcpyAsync(s.d_gather, s.h_gather, n_gather * sizeof(DevCopy), hipMemcpyHostToDevice, s.stream);
  if (e == hipSuccess && n_scatter)
    e = hipMemcpyAsync(s.d_scatter, s.h_scatter, n_scatter * sizeof(DevCopy), hipMemcpyHostToDevice, s.stream);
  if (e == hipSuccess && n_gather) {
    hipLaunchKernelGGL(k_srv_gather, dim3(n_gather < 2048 ? n_gather : 2048), dim3(256), 0, s.stream, s.d_gather,
                       n_gather, s.d_in);
    e = hipGetLastError();
  }
  utfx_status bs = UTFX_OK;
  if (e == hipSuccess)
    bs = utfx_batch_run(s.ctx, s.d_in, c.arena_in_bytes, s.d_out, c.arena_out_bytes, s.d_items, n, units, s.d_res);
  if (e == hipSuccess && bs == UTFX_OK)
    e = hipMemcpyAsync(s.h_res, s.d_res, n * sizeof(utfx_result), hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess && bs == UTFX_OK && out_lo)
    e = hipMemcpyAsync(s.h_out, s.d_out, out_lo, hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess && bs == UTFX_OK && n_scatter) {
    hipLaunchKernelGGL(k_srv_scatter, dim3(n_scatter < 2048 ? n_scatter : 2048), dim3(256), 0, s.stream,
                       s.d_scatter, n_scatter, s.d_out, s.d_res);
    e = hipGetLastError();
  }
  for (uint32_t k = 0; k < n && e == hipSuccess && bs == UTFX_OK; ++k) {
    if (s.direct_out[k] && !s.reqs[k].dev)
      e = hipMemcpyAsync(s.reqs[k].out, s.d_out + s.h_items[k].out_off, out_bytes(s.reqs[k]), hipMemcpyDeviceToHost,
                         s.stream);
  }
  if (e == hipSuccess && bs == UTFX_OK) e = hipEventRecord(s.done, s.stream);
  if (e != hipSuccess || bs != UTFX_OK) {
    snprintf(S->err, sizeof(S->err), "step launch: %s / status %d", hipGetErrorString(e), (int)bs);
    // copies already queued may still read the slot's staging buffers: let them end
    // before the slot takes another step
    (void)hipStreamSynchronize(s.stream);
    for (const Req& r : s.reqs) S->failed.add(r.tag);
    s.reqs.clear();
    return n;
  }
  s.busy = true;
  s.bulk = bulk;
  S->steps++;
  S->items_total += n;
  return n;
}

}  // namespace utfx_srv

extern "C" {

utfx_status utfx_server_create(utfx_server** out, const utfx_server_config* cfg) {
  using namespace utfx_srv;
  if (!out || !cfg || cfg->inflight < 1 || cfg->inflight > 16 || cfg->max_items < 1 || cfg->arena_in_bytes < 16 ||
      cfg->arena_out_bytes < 16)
    return UTFX_E_INVALID_ARG;
  *out = nullptr;
  const uint64_t dev = (uint64_t)cfg->inflight * (cfg->arena_in_bytes + cfg->arena_out_bytes);
  if (cfg->device_cap_bytes && dev > cfg->device_cap_bytes) return UTFX_E_INVALID_ARG;
  utfx_server* S = new (std::nothrow) utfx_server();
  if (!S) return UTFX_E_DEVICE;
  S->cfg = *cfg;
  S->err[0] = 0;
  S->slots.resize(cfg->inflight);
  for (auto& s : S->slots) {
    bool ok = alloc_slot(s, *cfg) == hipSuccess;
    // size the slot's batch workspace for any step now, so serving never allocates:
    // a step of max_items empty items with the largest possible input total
    if (ok) ok = hipMemsetAsync(s.d_items, 0, cfg->max_items * sizeof(utfx_item), s.stream) == hipSuccess;
    if (ok)
      ok = utfx_batch_run(s.ctx, s.d_in, cfg->arena_in_bytes, s.d_out, cfg->arena_out_bytes, s.d_items,
                          cfg->max_items, cfg->arena_in_bytes, s.d_res) == UTFX_OK;
    // and run every copy a step makes once, small and arena-sized, so that the runtime
    // sets up its copy engines now rather than inside the first steps that need them
    if (ok) ok = warm_copies(s, *cfg) == hipSuccess;
    if (ok) ok = hipStreamSynchronize(s.stream) == hipSuccess;
    if (!ok) {
      for (auto& t : S->slots) free_slot(t);
      delete S;
      return UTFX_E_DEVICE;
    }
  }
  *out = S;
  return UTFX_OK;
}

void utfx_server_destroy(utfx_server* S) {
  if (!S) return;
  for (auto& s : S->slots) utfx_srv::free_slot(s);
  delete S;
}

const char* utfx_server_last_error(const utfx_server* S) { return S ? S->err : "null server"; }

utfx_status utfx_server_submit(utfx_server* S, uint64_t tag, const void* data, uint64_t len_units, uint32_t dir,
                               void* out, uint64_t out_cap_units) {
  if (!S || (len_units && !data) || (out_cap_units && !out)) return UTFX_E_INVALID_ARG;
  const bool dev = (dir & UTFX_SERVER_DEVICE_BUFFERS) != 0;
  const utfx_srv::Req r{tag, static_cast<const uint8_t*>(data), len_units, dir & ~UTFX_SERVER_DEVICE_BUFFERS,
                        static_cast<uint8_t*>(out), out_cap_units, dev};
  (utfx_srv::in_bytes(r) >= utfx_srv::kBulkMin ? S->pending_bulk : S->pending).push_back(r);
  return UTFX_OK;
}

utfx_status utfx_server_progress(utfx_server* S, utfx_completion* done, uint32_t max_done, uint32_t* n_done) {
  using namespace utfx_srv;
  if (!S || !n_done || (max_done && !done)) return UTFX_E_INVALID_ARG;
  *n_done = 0;
  utfx_status st = UTFX_OK;
  // completions first (a slot is only drained when all its requests fit in `done`)
  for (auto& s : S->slots) {
    if (!s.busy || *n_done + s.reqs.size() > max_done) continue;
    const hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) {
      snprintf(S->err, sizeof(S->err), "step: %s", hipGetErrorString(q));
      return UTFX_E_DEVICE;
    }
    for (size_t i = 0; i < s.reqs.size(); ++i) {
      const Req& r = s.reqs[i];
      const utfx_result& res = s.h_res[i];
      const uint64_t w = res.written < r.out_cap ? res.written : r.out_cap;
      const uint64_t ob = w * (r.dir ? 1 : 2);
      if (ob && res.status != UTFX_E_OUTPUT_TOO_SMALL && !s.direct_out[i])
        memcpy(r.out, s.h_out + s.h_items[i].out_off, ob);
      utfx_completion& c = done[(*n_done)++];
      c.tag = r.tag;
      c.result = res;
    }
    s.busy = false;
    s.reqs.clear();
  }
  // requests no slot can hold, and requests of steps that could not be launched
  while (!S->rejected.empty() && *n_done < max_done) {
    utfx_completion& c = done[(*n_done)++];
    c.tag = S->rejected.front();
    c.result.status = UTFX_E_INVALID_ARG;
    c.result.reserved = 0;
    c.result.count = 0;
    c.result.written = 0;
    S->rejected.pop_front();
  }
  while (!S->failed.empty() && *n_done < max_done) {
    utfx_completion& c = done[(*n_done)++];
    c.tag = S->failed.pop();
    c.result.status = UTFX_E_DEVICE;
    c.result.reserved = 0;
    c.result.count = 0;
    c.result.written = 0;
  }
  // then launch steps on free slots while requests wait: a bulk step when none is in
  // flight, small steps otherwise, and more bulk steps only while no small request
  // waits
  bool bulk_busy = false;
  for (auto& s : S->slots) bulk_busy |= s.busy && s.bulk;
  for (auto& s : S->slots) {
    if (s.busy) continue;
    const int which = pick_queue(!S->pending_bulk.empty(), !S->pending.empty(), bulk_busy);
    if (which == 1) {
      launch_step(S, s, S->pending_bulk, true);
      bulk_busy = s.busy;
    } else if (which == 0) {
      launch_step(S, s, S->pending, false);
    }
  }
  return st;
}

utfx_status utfx_server_replay(utfx_server* S, uint32_t n, const uint64_t* arrival_ns, const void* const* data,
                               const uint64_t* len_units, const uint32_t* dirs, void* const* outs,
                               const uint64_t* out_caps, uint64_t* latency_ns, utfx_result* results,
                               uint64_t* wall_ns) {
  using namespace utfx_srv;
  if (!S || (n && (!arrival_ns || !data || !len_units || !dirs || !outs || !out_caps || !latency_ns || !results)))
    return UTFX_E_INVALID_ARG;
  std::vector<utfx_completion> done(S->cfg.max_items * S->slots.size() + 64);
  const uint64_t t0 = now_ns();
  uint32_t next = 0, finished = 0;
  while (finished < n) {
    uint64_t t = now_ns() - t0;
    while (next < n && arrival_ns[next] <= t) {
      utfx_server_submit(S, next, data[next], len_units[next], dirs[next], outs[next], out_caps[next]);
      ++next;
    }
    uint32_t k = 0;
    utfx_status st = utfx_server_progress(S, done.data(), (uint32_t)done.size(), &k);
    if (st != UTFX_OK) return st;
    if (k) {
      t = now_ns() - t0;
      for (uint32_t j = 0; j < k; ++j) {
        const uint64_t i = done[j].tag;
        results[i] = done[j].result;
        latency_ns[i] = t - arrival_ns[i];
      }
      finished += k;
    }
  }
  if (wall_ns) *wall_ns = now_ns() - t0;
  return UTFX_OK;
}

}  // extern "C"
