// utfx.hip -- host runtime and C ABI of libutfx.so (see include/utfx.h).
//
// The context owns a device workspace (a 64-byte header of counters and a status
// word per segment for the look-back, STATUS_STRIDE words apart), a device result slot and a pinned host copy of
// it.  A call checks its arguments, sizes the grid, launches one kernel on the
// context's stream and, for the synchronous entry points, copies the 24-byte result
// back.  Kernels reset the workspace counters themselves (the last workgroup of every
// launch does it), so no call issues a memset and launches can be graph-captured.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "utfx.h"
#include "utfx_kernels.hpp"
#include "utfx_transcode.hpp"
#include "utfx_batch.hpp"
#include "utfx_stream.hpp"
#include "utfx_utf32.hpp"

using namespace utfx_dev;

static_assert(sizeof(utfx_result) == 24, "utfx_result layout");
static_assert(sizeof(Result) == sizeof(utfx_result), "device result layout");
static_assert(sizeof(WsHeader) == 64, "workspace header layout");
static_assert(sizeof(utfx_stream) == 48 && offsetof(utfx_stream, carry) == 40 && offsetof(utfx_stream, carry_need) == 44,
              "stream state layout");
static_assert(sizeof(utfx_item) == sizeof(BItem) && offsetof(utfx_item, dir) == offsetof(BItem, dir), "item layout");

struct utfx_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cus = 256;
  uint32_t cu_lds = 160u << 10;           // LDS bytes of one CU
  WsHeader* ws = nullptr;                 // device header
  unsigned long long* status = nullptr;   // device status words
  uint64_t cap_tiles = 0;
  Result* d_result = nullptr;             // device result slot of synchronous calls
  Result* h_result = nullptr;             // pinned host slot the finalisation kernels write directly
  Result* h_result_dev = nullptr;         // the same memory as the device addresses it (null: copy instead)
  StreamDev* d_stream = nullptr;          // stream calls: staged character and its output
  StreamRec* h_stream = nullptr;          // stream calls: results and cut, written by the kernels (pinned)
  StreamRec* h_stream_dev = nullptr;      // the same memory as the device addresses it
  uint64_t launches = 0;                  // launches since the status words were cleared
  uint32_t tile_bytes[UTFX_OP_COUNT_];
  uint32_t seg_tiles[UTFX_OP_COUNT_];
  uint32_t wgs_per_cu[UTFX_OP_COUNT_];
  BatchWs batch;                          // batched-path workspace
  BatchTuning batch_tuning;               // utfx_set_batch_tuning
  // graph capture: while capturing, calls are recorded on cap_stream
  bool capturing = false;
  hipStream_t user_stream = nullptr;
  hipStream_t cap_stream = nullptr;
  uint64_t cap_launches = 0;              // single-buffer launches recorded so far
  uint64_t cap_batches = 0;               // batched calls recorded so far
  // generation of the workspace memory: bumped whenever the single-buffer or the
  // batch workspace is reallocated, so that a graph holding the old addresses is refused
  uint64_t ws_gen = 0;
  uint32_t dbg = 0;                       // look-back delay injection (UTFX_DEBUG_LOOKBACK_DELAY)
  hipEvent_t kev_start = nullptr;         // kernel timing events (utfx_set_kernel_events)
  hipEvent_t kev_stop = nullptr;
  char err[256];
};

// Workspace of the allocation-free call (utfx_utf8_to_utf16le_noalloc): a workspace
// header and one status word per segment of 32 KiB, STATUS_STRIDE words apart.  Each
// device holds its own copy for the life of the process.
constexpr uint32_t kNoAllocWg = 512, kNoAllocSeg = 4;
constexpr uint64_t kNoAllocSegUnits = 16ull * kNoAllocWg * kNoAllocSeg;
constexpr uint64_t kNoAllocSegs = 16384;
constexpr uint64_t kNoAllocWords = sizeof(WsHeader) / 8 + kNoAllocSegs * STATUS_STRIDE;
static_assert(UTFX_NOALLOC_MAX_BYTES + 15 + 1 <= kNoAllocSegs * kNoAllocSegUnits, "scratch covers the size limit");
static_assert(sizeof(WsHeader) % 8 == 0, "header in whole words");

static __device__ __align__(256) unsigned long long scratch[kNoAllocWords];

struct utfx_graph {
  utfx_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t launches = 0;                  // single-buffer launches per replay
  uint64_t batches = 0;                   // batched calls per replay
  uint64_t ws_gen = 0;                    // workspace generation the kernels' addresses belong to
};

namespace {

constexpr uint64_t kInitialTiles = 1ull << 20;
constexpr uint64_t kEpochClearEvery = 1ull << 24;  // well inside the 25-bit epoch space

utfx_result mkres(int32_t st, uint64_t count, uint64_t written) {
  utfx_result r;
  r.status = st;
  r.reserved = 0;
  r.count = count;
  r.written = written;
  return r;
}

void set_err(utfx_ctx* c, const char* what, hipError_t e) {
  if (!c) return;
  snprintf(c->err, sizeof(c->err), "%s: %s", what, hipGetErrorString(e));
}

void set_msg(utfx_ctx* c, const char* what) {
  if (!c) return;
  snprintf(c->err, sizeof(c->err), "%s", what);
}

// (Re)initialises the header and clears every status word.  Synchronous.
utfx_status init_ws(utfx_ctx* c) {
  hipError_t e = hipMemsetAsync(c->status, 0, c->cap_tiles * STATUS_STRIDE * sizeof(unsigned long long), c->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(64), 0, c->stream, c->ws);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    set_err(c, "workspace init", e);
    return UTFX_E_DEVICE;
  }
  c->launches = 0;
  return UTFX_OK;
}

utfx_status alloc_ws(utfx_ctx* c, uint64_t tiles) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(WsHeader) + tiles * STATUS_STRIDE * sizeof(unsigned long long));
  if (e != hipSuccess) {
    set_err(c, "workspace allocation", e);
    return UTFX_E_DEVICE;
  }
  c->ws = reinterpret_cast<WsHeader*>(p);
  c->status = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(p) + sizeof(WsHeader));
  c->cap_tiles = tiles;
  c->ws_gen++;
  return init_ws(c);
}

// Makes room for `tiles` status words.  Growing synchronises the stream once; a
// workload of a fixed size never grows again.
utfx_status ensure_tiles(utfx_ctx* c, uint64_t tiles) {
  if (c->capturing && (c->launches >= kEpochClearEvery || tiles > c->cap_tiles)) {
    set_msg(c, "workspace must grow during graph capture; make the same call once before capturing");
    return UTFX_E_INVALID_ARG;
  }
  if (c->launches >= kEpochClearEvery) {
    utfx_status s = init_ws(c);
    if (s != UTFX_OK) return s;
  }
  if (tiles <= c->cap_tiles) return UTFX_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    set_err(c, "stream sync", e);
    return UTFX_E_DEVICE;
  }
  (void)hipFree(c->ws);
  c->ws = nullptr;
  c->status = nullptr;
  uint64_t want = c->cap_tiles;
  while (want < tiles) want *= 2;
  return alloc_ws(c, want);
}

bool valid_tile(uint32_t t) { return t == 4096 || t == 8192; }

// Common launch geometry: base rounded down to 16 bytes, misalignment in units,
// tiles covering logical positions [-mis, n + extra).
// Launch description for a kernel of wg_ threads and seg_tiles tiles per segment.
utfx_status prep_cfg(utfx_ctx* c, uint32_t wg_, uint32_t seg_tiles, const void* in, uint64_t n, uint32_t unit,
                     uint64_t extra, void* result, Launch& L, uint32_t& wg) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(in);
  L.base = reinterpret_cast<const uint8_t*>(a & ~static_cast<uintptr_t>(15));
  L.mis = (a & 15) / unit;
  L.n = n;
  wg = wg_;
  L.seg = seg_tiles;
  L.wg = wg;
  L.be = 0;
  L.dbg = c->dbg;
  const uint64_t per_seg = static_cast<uint64_t>(wg) * (16 / unit) * L.seg;
  L.seg_units = per_seg;
  L.ntiles = (L.mis + n + extra + per_seg - 1) / per_seg;
  utfx_status s = ensure_tiles(c, L.ntiles);
  if (s != UTFX_OK) return s;
  L.ws = c->ws;
  L.err = &c->ws->err;
  L.status = c->status;
  L.result = result;
  L.out = nullptr;
  L.cap = 0;
  return UTFX_OK;
}

utfx_status prep(utfx_ctx* c, int op, const void* in, uint64_t n, uint32_t unit, uint64_t extra,
                 void* result, Launch& L, uint32_t& wg) {
  return prep_cfg(c, c->tile_bytes[op] / 16, c->seg_tiles[op], in, n, unit, extra, result, L, wg);
}

template <template <int> class K>
struct Launcher;

#define UTFX_DEFINE_LAUNCH(NAME, KERNEL)                                                         \
  hipError_t NAME(uint32_t wg, uint64_t grid, const Launch& L, hipStream_t s) {                 \
    switch (wg) {                                                                               \
      case 256: UTFX_KLAUNCH(KERNEL<256>, dim3((uint32_t)grid), 256, s, L); break; \
      default: UTFX_KLAUNCH(KERNEL<512>, dim3((uint32_t)grid), 512, s, L); break; \
    }                                                                                           \
    return hipGetLastError();                                                                   \
  }

// Events recorded around the main kernel of the call being launched (hipExtLaunchKernel
// records them on the stream immediately before and after that kernel); null when the
// context has none or is capturing.  Set by run() for the duration of one launch.
thread_local hipEvent_t t_kev_start = nullptr, t_kev_stop = nullptr;

// Residency cap of the launch being made (workgroups per CU, 0 = none) and the LDS of
// one CU; set by run() like the events.
thread_local uint32_t t_wgs_per_cu = 0;
thread_local uint32_t t_cu_lds = 0;

// Dynamic LDS (unused by the kernel) that caps its residency at `wgs` workgroups per
// CU: with it, one workgroup takes more than 1/(wgs + 1) of the CU's LDS, so at most
// wgs fit.  0 when wgs is 0 or the kernel's own LDS already allows no more.  The
// kernel's static LDS is looked up once per kernel.
uint32_t lds_pad(const void* kernel, uint32_t wgs, uint32_t cu_lds) {
  if (!wgs || !cu_lds) return 0;
  static std::mutex mu;
  static const void* keys[64];
  static uint32_t vals[64];
  static int nk = 0;
  uint32_t stat = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    int i = 0;
    while (i < nk && keys[i] != kernel) ++i;
    if (i == nk) {
      hipFuncAttributes a;
      if (hipFuncGetAttributes(&a, kernel) != hipSuccess) return 0;
      if (nk < 64) {
        keys[nk] = kernel;
        vals[nk] = (uint32_t)a.sharedSizeBytes;
        ++nk;
      }
      stat = (uint32_t)a.sharedSizeBytes;
    } else {
      stat = vals[i];
    }
  }
  const uint32_t need = ((cu_lds / (wgs + 1) + 1) + 511) & ~511u;
  return need > stat ? need - stat : 0;
}

#define UTFX_KLAUNCH(K, GRID, WG, S, L)                                                                   \
  hipExtLaunchKernelGGL(K, GRID, dim3(WG), lds_pad(reinterpret_cast<const void*>(&K), t_wgs_per_cu, t_cu_lds), \
                        S, t_kev_start, t_kev_stop, 0, L)

UTFX_DEFINE_LAUNCH(launch_len8, k_len8)
UTFX_DEFINE_LAUNCH(launch_len16, k_len16)
UTFX_DEFINE_LAUNCH(launch_val8, k_validate8)
UTFX_DEFINE_LAUNCH(launch_val16, k_validate16)

// Transcode kernels are instantiated per (workgroup size, tiles per segment); a whole
// segment's output is staged in LDS (up to 96 KiB of the 160 KiB a gfx950 workgroup
// may use).
#define UTFX_LAUNCH_WS(K, WG, S) UTFX_KLAUNCH((K<WG, S>), g, WG, s, L)

hipError_t launch_u8u16(uint32_t wg, uint64_t grid, const Launch& L, hipStream_t s) {
  const dim3 g((uint32_t)grid);
  if (wg == 256) {
    if (L.seg == 2) UTFX_LAUNCH_WS(k_u8_to_u16, 256, 2);
    else if (L.seg == 4) UTFX_LAUNCH_WS(k_u8_to_u16, 256, 4);
    else UTFX_LAUNCH_WS(k_u8_to_u16, 256, 8);
  } else {
    if (L.seg == 2) UTFX_LAUNCH_WS(k_u8_to_u16, 512, 2);
    else UTFX_LAUNCH_WS(k_u8_to_u16, 512, 4);
  }
  return hipGetLastError();
}

hipError_t launch_u16u8(uint32_t wg, uint64_t grid, const Launch& L, hipStream_t s) {
  const dim3 g((uint32_t)grid);
  if (wg == 256) {
    if (L.seg == 2) UTFX_LAUNCH_WS(k_u16_to_u8, 256, 2);
    else if (L.seg == 4) UTFX_LAUNCH_WS(k_u16_to_u8, 256, 4);
    else UTFX_LAUNCH_WS(k_u16_to_u8, 256, 8);
  } else {
    if (L.seg == 2) UTFX_LAUNCH_WS(k_u16_to_u8, 512, 2);
    else if (L.seg == 4) UTFX_LAUNCH_WS(k_u16_to_u8, 512, 4);
    else UTFX_LAUNCH_WS(k_u16_to_u8, 512, 8);
  }
  return hipGetLastError();
}

// (tile bytes, tiles per segment) pairs with a transcode kernel instance
bool transcode_config_ok(int op, uint32_t tile_bytes, uint32_t seg) {
  if (op == UTFX_OP_UTF8_TO_UTF16)
    return (tile_bytes == 4096 && (seg == 2 || seg == 4 || seg == 8)) || (tile_bytes == 8192 && (seg == 2 || seg == 4));
  if (op == UTFX_OP_UTF16_TO_UTF8)
    return (seg == 2 || seg == 4 || seg == 8) && (tile_bytes == 4096 || tile_bytes == 8192);
  return true;
}

hipError_t launch_fin_u8u16(uint32_t wg, const Launch& L, hipStream_t s) {
  if (wg == 256) hipLaunchKernelGGL(k_fin_u8u16<256>, dim3(1), dim3(256), 0, s, L);
  else hipLaunchKernelGGL(k_fin_u8u16<512>, dim3(1), dim3(512), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_fin_u16u8(uint32_t wg, const Launch& L, hipStream_t s) {
  if (wg == 256) hipLaunchKernelGGL(k_fin_u16u8<256>, dim3(1), dim3(256), 0, s, L);
  else hipLaunchKernelGGL(k_fin_u16u8<512>, dim3(1), dim3(512), 0, s, L);
  return hipGetLastError();
}

// One-workgroup finalisation that follows every main launch on the same stream.
hipError_t launch_fin(int kind, uint32_t wg, const Launch& L, hipStream_t s);

__global__ void k_store_result(Result* r, int32_t st, uint64_t count, uint64_t written) {
  if (threadIdx.x == 0) {
    r->status = st;
    r->reserved = 0;
    r->count = count;
    r->written = written;
  }
}

utfx_status store_result_async(utfx_ctx* c, void* d_result, int32_t st, uint64_t count, uint64_t written) {
  hipLaunchKernelGGL(k_store_result, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<Result*>(d_result), st,
                     count, written);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_err(c, "result launch", e);
    return UTFX_E_DEVICE;
  }
  return UTFX_OK;
}

enum Kind { LEN8, LEN16, VAL8, VAL16, U8U16, U16U8, VAL32, U8U32, U32U8, U16U32, U32U16 };

// UTF-32 launches use one fixed configuration each: (threads, tiles per segment), the
// fastest of 2, 4 and 8 tiles measured on 256 MiB inputs.
constexpr uint32_t kU8U32Wg = 256, kU8U32Seg = 2, kU32U8Wg = 256, kU32U8Seg = 4, kVal32Wg = 256, kVal32Seg = 8;
constexpr uint32_t kU16U32Wg = 256, kU16U32Seg = 4, kU32U16Wg = 256, kU32U16Seg = 8;

hipError_t launch_fin(int kind, uint32_t wg, const Launch& L, hipStream_t s) {
  switch (kind) {
    case LEN8:
    case LEN16:
      hipLaunchKernelGGL(k_fin_len<512>, dim3(1), dim3(512), 0, s, L);
      return hipGetLastError();
    case VAL8:
      hipLaunchKernelGGL(k_fin_validate8, dim3(1), dim3(64), 0, s, L);
      return hipGetLastError();
    case VAL16:
      hipLaunchKernelGGL(k_fin_validate16, dim3(1), dim3(64), 0, s, L);
      return hipGetLastError();
    case U8U16:
      return launch_fin_u8u16(wg, L, s);
    case VAL32:
      hipLaunchKernelGGL(k_fin_validate32, dim3(1), dim3(64), 0, s, L);
      return hipGetLastError();
    case U8U32:
      hipLaunchKernelGGL(k_fin_u8u32<kU8U32Wg>, dim3(1), dim3(kU8U32Wg), 0, s, L);
      return hipGetLastError();
    case U32U8:
      hipLaunchKernelGGL((k_fin_u32to<kU32U8Wg, false>), dim3(1), dim3(kU32U8Wg), 0, s, L);
      return hipGetLastError();
    case U32U16:
      hipLaunchKernelGGL((k_fin_u32to<kU32U16Wg, true>), dim3(1), dim3(kU32U16Wg), 0, s, L);
      return hipGetLastError();
    case U16U32:
      hipLaunchKernelGGL(k_fin_u16u32<kU16U32Wg>, dim3(1), dim3(kU16U32Wg), 0, s, L);
      return hipGetLastError();
    default:
      return launch_fin_u16u8(wg, L, s);
  }
}

// be: the UTF-16 side (input or output) is big-endian.
utfx_status run(utfx_ctx* c, Kind kind, const void* in, uint64_t n, void* out, uint64_t cap, void* d_result,
                bool be = false) {
  if (!c) return UTFX_E_INVALID_ARG;
  c->err[0] = 0;
  const bool in16 = (kind == LEN16 || kind == VAL16 || kind == U16U8 || kind == U16U32);
  const bool out16 = (kind == U8U16 || kind == U32U16);
  const bool in32 = (kind == VAL32 || kind == U32U8 || kind == U32U16);
  const bool out32 = (kind == U8U32 || kind == U16U32);
  const bool has_out = (kind == U8U16 || kind == U16U8 || kind == U8U32 || kind == U32U8 || kind == U16U32 ||
                        kind == U32U16);
  if (!d_result) {
    set_msg(c, "null result pointer");
    return UTFX_E_INVALID_ARG;
  }
  if (n > 0 && !in) {
    set_msg(c, "null input with n > 0");
    return UTFX_E_INVALID_ARG;
  }
  if (n > UTFX_MAX_UNITS) {
    set_msg(c, "input longer than UTFX_MAX_UNITS");
    return UTFX_E_INVALID_ARG;
  }
  if (in16 && (reinterpret_cast<uintptr_t>(in) & 1)) {
    set_msg(c, "UTF-16 input not 2-byte aligned");
    return UTFX_E_INVALID_ARG;
  }
  if (has_out && cap > 0 && !out) {
    set_msg(c, "null output with cap > 0");
    return UTFX_E_INVALID_ARG;
  }
  if (out16 && (reinterpret_cast<uintptr_t>(out) & 1)) {
    set_msg(c, "UTF-16 output not 2-byte aligned");
    return UTFX_E_INVALID_ARG;
  }
  if (in32 && (reinterpret_cast<uintptr_t>(in) & 3)) {
    set_msg(c, "UTF-32 input not 4-byte aligned");
    return UTFX_E_INVALID_ARG;
  }
  if (out32 && (reinterpret_cast<uintptr_t>(out) & 3)) {
    set_msg(c, "UTF-32 output not 4-byte aligned");
    return UTFX_E_INVALID_ARG;
  }
  if (n == 0) return store_result_async(c, d_result, UTFX_OK, 0, 0);

  int op = 0;
  uint32_t unit = in32 ? 4 : (in16 ? 2 : 1);
  uint64_t extra = 0;
  switch (kind) {
    case VAL32:
    case U8U32:
    case U32U8:
    case U16U32:
    case U32U16: break;
    case LEN8: op = UTFX_OP_LENGTH_UTF8; break;
    case LEN16: op = UTFX_OP_LENGTH_UTF16; break;
    case VAL8: op = UTFX_OP_VALIDATE_UTF8; extra = 1; break;
    case VAL16: op = UTFX_OP_VALIDATE_UTF16; extra = 1; break;
    case U8U16: op = UTFX_OP_UTF8_TO_UTF16; extra = 1; break;
    case U16U8: op = UTFX_OP_UTF16_TO_UTF8; extra = 1; break;
  }
  Launch L;
  uint32_t wg = 0;
  utfx_status s;
  if (kind == VAL32) s = prep_cfg(c, kVal32Wg, kVal32Seg, in, n, unit, 0, d_result, L, wg);
  else if (kind == U8U32) s = prep_cfg(c, kU8U32Wg, kU8U32Seg, in, n, unit, 1, d_result, L, wg);
  else if (kind == U32U8) s = prep_cfg(c, kU32U8Wg, kU32U8Seg, in, n, unit, 0, d_result, L, wg);
  else if (kind == U16U32) s = prep_cfg(c, kU16U32Wg, kU16U32Seg, in, n, unit, 1, d_result, L, wg);
  else if (kind == U32U16) s = prep_cfg(c, kU32U16Wg, kU32U16Seg, in, n, unit, 0, d_result, L, wg);
  else s = prep(c, op, in, n, unit, extra, d_result, L, wg);
  if (s != UTFX_OK) return s;
  L.out = out;
  L.cap = cap;
  L.be = be ? 1u : 0u;
  if (L.ntiles > 0x7FFFFFFFull) {
    set_msg(c, "grid too large");
    return UTFX_E_INVALID_ARG;
  }
  hipError_t e = hipSuccess;
  if (!c->capturing) {
    t_kev_start = c->kev_start;
    t_kev_stop = c->kev_stop;
  }
  t_wgs_per_cu = (kind == LEN8 || kind == LEN16 || kind == VAL8 || kind == VAL16 || kind == U8U16 || kind == U16U8)
                     ? c->wgs_per_cu[op]
                     : 0u;
  t_cu_lds = c->cu_lds;
  switch (kind) {
    case LEN8: e = launch_len8(wg, L.ntiles, L, c->stream); break;
    case LEN16: e = launch_len16(wg, L.ntiles, L, c->stream); break;
    case VAL8: e = launch_val8(wg, L.ntiles, L, c->stream); break;
    case VAL16: e = launch_val16(wg, L.ntiles, L, c->stream); break;
    case U8U16: e = launch_u8u16(wg, L.ntiles, L, c->stream); break;
    case U16U8: e = launch_u16u8(wg, L.ntiles, L, c->stream); break;
    case VAL32:
      UTFX_KLAUNCH(k_validate32<kVal32Wg>, dim3((uint32_t)L.ntiles), kVal32Wg, c->stream, L);
      e = hipGetLastError();
      break;
    case U8U32:
      UTFX_KLAUNCH((k_u8_to_u32<kU8U32Wg, kU8U32Seg>), dim3((uint32_t)L.ntiles), kU8U32Wg, c->stream, L);
      e = hipGetLastError();
      break;
    case U32U8:
      UTFX_KLAUNCH((k_u32_to<kU32U8Wg, kU32U8Seg, uint8_t>), dim3((uint32_t)L.ntiles), kU32U8Wg, c->stream, L);
      e = hipGetLastError();
      break;
    case U32U16:
      UTFX_KLAUNCH((k_u32_to<kU32U16Wg, kU32U16Seg, uint16_t>), dim3((uint32_t)L.ntiles), kU32U16Wg, c->stream,
                   L);
      e = hipGetLastError();
      break;
    case U16U32:
      UTFX_KLAUNCH((k_u16_to_u32<kU16U32Wg, kU16U32Seg>), dim3((uint32_t)L.ntiles), kU16U32Wg, c->stream, L);
      e = hipGetLastError();
      break;
  }
  t_kev_start = t_kev_stop = nullptr;
  t_wgs_per_cu = 0;
  if (e == hipSuccess) e = launch_fin(kind, wg, L, c->stream);
  if (e != hipSuccess) {
    set_err(c, "kernel launch", e);
    return UTFX_E_DEVICE;
  }
  c->launches++;
  if (c->capturing) c->cap_launches++;
  return UTFX_OK;
}

utfx_result run_sync(utfx_ctx* c, Kind kind, const void* in, uint64_t n, void* out, uint64_t cap,
                     bool be = false) {
  if (!c) return mkres(UTFX_E_INVALID_ARG, 0, 0);
  if (c->capturing) {
    set_msg(c, "synchronous call during graph capture");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  // the finalisation kernel writes the result straight into pinned host memory when the
  // device can address it (saves a copy per call), else into a device slot copied back
  utfx_status s = run(c, kind, in, n, out, cap, c->h_result_dev ? static_cast<void*>(c->h_result_dev) : c->d_result,
                      be);
  if (s != UTFX_OK) return mkres(s, 0, 0);
  hipError_t e = hipSuccess;
  if (!c->h_result_dev)
    e = hipMemcpyAsync(c->h_result, c->d_result, sizeof(Result), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    set_err(c, "synchronise", e);
    return mkres(UTFX_E_DEVICE, 0, 0);
  }
  utfx_result r;
  memcpy(&r, c->h_result, sizeof(r));
  if (r.status == UTFX_E_DEVICE) {
    set_msg(c, "look-back watchdog fired; workspace reinitialised");
    init_ws(c);
  }
  return r;
}

bool encoding_error(int32_t st) { return st >= UTFX_E_STRAY_CONT && st <= UTFX_E_BAD_BYTE; }

// One stream call: k_stream_edge stages and transcodes the character across the cut
// (piece 1) and finds the unfinished one at the chunk's end, piece 2 (the rest of the
// chunk, in place) runs as an ordinary single-buffer transcode, and one copy brings
// everything back.  The host does offsets only; every unit is looked at on the
// device.
utfx_result stream_transcode(utfx_ctx* c, utfx_stream* st, const void* in, uint64_t n, void* out, uint64_t cap,
                             bool final) {
  if (!c) return mkres(UTFX_E_INVALID_ARG, 0, 0);
  c->err[0] = 0;
  if (!st || st->format < UTFX_STREAM_UTF8_TO_UTF16LE || st->format > UTFX_STREAM_UTF16BE_TO_UTF8) {
    set_msg(c, "null or malformed stream state");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  const bool in16 = (st->format == UTFX_STREAM_UTF16LE_TO_UTF8 || st->format == UTFX_STREAM_UTF16BE_TO_UTF8);
  const bool be = (st->format == UTFX_STREAM_UTF8_TO_UTF16BE || st->format == UTFX_STREAM_UTF16BE_TO_UTF8);
  if (st->status != UTFX_OK) {
    if (!encoding_error(st->status)) {
      set_msg(c, "malformed stream state");
      return mkres(UTFX_E_INVALID_ARG, 0, 0);
    }
    return mkres(st->status, st->err_offset, 0);
  }
  if (st->finished) {
    set_msg(c, "stream already finished");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  const uint32_t nc = st->n_carry;
  if (nc > (in16 ? 1u : 3u) || (nc > 0) != (st->carry_need > 0) || st->carry_need > 3 || st->carry_out > 4) {
    set_msg(c, "malformed stream state");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  if (c->capturing) {
    set_msg(c, "synchronous call during graph capture");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  if (n > 0 && !in) {
    set_msg(c, "null input with n > 0");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  if (n > UTFX_MAX_UNITS) {
    set_msg(c, "input longer than UTFX_MAX_UNITS");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  if (in16 && (reinterpret_cast<uintptr_t>(in) & 1)) {
    set_msg(c, "UTF-16 input not 2-byte aligned");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  if (cap > 0 && !out) {
    set_msg(c, "null output with cap > 0");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  if (!in16 && (reinterpret_cast<uintptr_t>(out) & 1)) {
    set_msg(c, "UTF-16 output not 2-byte aligned");
    return mkres(UTFX_E_INVALID_ARG, 0, 0);
  }
  if (n == 0 && nc == 0) {
    if (final) st->finished = 1;
    return mkres(UTFX_OK, 0, 0);
  }
  const uint64_t h = nc ? (n < st->carry_need ? n : st->carry_need) : 0;
  const bool grow = nc && !final && h < st->carry_need;  // the chunk does not finish the carried character
  uint32_t carry = 0;
  memcpy(&carry, st->carry, 4);
  const uint32_t flags = (in16 ? SE_IN16 : 0u) | (be ? SE_BE : 0u) | (final ? SE_FINAL : 0u);
  hipLaunchKernelGGL(k_stream_edge, dim3(1), dim3(64), 0, c->stream, c->d_stream, c->h_stream_dev, in, n, h, carry,
                     nc, flags, grow ? 1u : 0u, out, cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_err(c, "stream edge launch", e);
    return mkres(UTFX_E_DEVICE, 0, 0);
  }
  const Kind kind = in16 ? U16U8 : U8U16;
  const uint64_t iu = in16 ? 2 : 1, ou = in16 ? 1 : 2;
  const bool p1 = nc > 0 && !grow, p2 = !grow && n > h;
  const uint64_t w1 = p1 ? st->carry_out : 0;  // piece 2's output starts after piece 1's
  const uint64_t cap2 = cap > w1 ? cap - w1 : 0;
  if (p2) {
    void* out2 = cap2 ? static_cast<void*>(static_cast<uint8_t*>(out) + w1 * ou) : nullptr;
    utfx_status s = run(c, kind, static_cast<const uint8_t*>(in) + h * iu, n - h, out2, cap2, &c->h_stream_dev->r[1], be);
    if (s != UTFX_OK) return mkres(s, 0, 0);
  }
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    set_err(c, "synchronise", e);
    return mkres(UTFX_E_DEVICE, 0, 0);
  }
  const StreamEdge cut = c->h_stream->e;
  Result r1{UTFX_OK, 0, 0, 0}, r2{UTFX_OK, 0, 0, 0};
  if (p1) r1 = c->h_stream->r[0];
  if (p2) r2 = c->h_stream->r[1];
  if (r1.status == UTFX_E_DEVICE || r2.status == UTFX_E_DEVICE) {
    set_msg(c, "look-back watchdog fired; workspace reinitialised");
    init_ws(c);
    return mkres(UTFX_E_DEVICE, 0, 0);
  }
  if (cut.t > n || cut.t < (grow ? n : h) || cut.n_keep != (grow ? nc + h : n - cut.t) ||
      cut.n_keep > (in16 ? 1u : 3u) || cut.keep_need > 3 || cut.keep_out > 4 || (cut.n_keep > 0) != (cut.keep_need > 0)) {
    set_msg(c, "stream cut out of range");
    return mkres(UTFX_E_DEVICE, 0, 0);
  }
  if (p2 && cut.t < n && encoding_error(r2.status) && r2.count == cut.t - h) {
    // the only error is the unfinished character at the end, which is carried: piece 2
    // is chunk[h, t), whose output is complete
    r2.status = r2.written > cap2 ? UTFX_E_OUTPUT_TOO_SMALL : UTFX_OK;
    r2.count = r2.written;
    if (r2.status != UTFX_OK) r2.written = 0;
  }
  const uint64_t base = st->in_units;  // stream offset of the chunk's first unit
  if (encoding_error(r1.status) || encoding_error(r2.status)) {
    utfx_result r;
    if (encoding_error(r1.status)) {
      r = mkres(r1.status, base - nc + r1.count, r1.written);
    } else {
      r = mkres(r2.status, base + h + r2.count, w1 + r2.written);
    }
    st->status = r.status;
    st->err_offset = r.count;
    st->in_units = base + n;
    st->out_units += r.written;
    st->n_carry = 0;
    st->carry_need = 0;
    st->carry_out = 0;
    return r;
  }
  // piece 2 was placed after w1 output units: piece 1 must have needed exactly that many
  if (p1 && r1.count != w1) {
    set_msg(c, "stream state disagrees with the staged character");
    return mkres(UTFX_E_DEVICE, 0, 0);
  }
  const uint64_t total = r1.count + r2.count;  // OK: units written; OUTPUT_TOO_SMALL: units needed
  if (r1.status == UTFX_E_OUTPUT_TOO_SMALL || r2.status == UTFX_E_OUTPUT_TOO_SMALL)
    return mkres(UTFX_E_OUTPUT_TOO_SMALL, total, 0);
  st->in_units = base + n;
  st->out_units += total;
  st->n_carry = cut.n_keep;
  memcpy(st->carry, cut.keep, 4);
  st->carry_need = static_cast<uint8_t>(cut.keep_need);
  st->carry_out = static_cast<uint8_t>(cut.keep_out);
  if (final) st->finished = 1;
  return mkres(UTFX_OK, total, total);
}

// ---------------------------------------------------------------- allocation-free call
//
// utfx_utf8_to_utf16le_noalloc runs the kernels of utfx_utf8_to_utf16le_async with its
// workspace in the file-scope array `scratch` (a workspace header and one status word per segment,
// STATUS_STRIDE words apart) instead of a context's.  Host code never passes the
// array's name to a kernel: it looks up the array's device address once per device
// (hipGetSymbolAddress, with that device current) and passes that.

// Clears the status words and initialises the header (the k_ws_init state), as one
// ordinary kernel so that a graph may record it.
__global__ void k_noalloc_clear(unsigned long long* words, uint64_t n_words) {
  const uint64_t hdr = sizeof(WsHeader) / 8;
  for (uint64_t i = hdr + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_words;
       i += (uint64_t)gridDim.x * blockDim.x)
    words[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    WsHeader* ws = reinterpret_cast<WsHeader*>(words);
    ws->spare0 = 0;
    ws->spare1 = 0;
    ws->err = NO_ERR;
    ws->acc = 0;
    ws->epoch = 1;
    ws->fault = 0;
  }
}

constexpr int kNoAllocMaxDevices = 64;
struct NoAllocDevice {
  unsigned long long* ptr = nullptr;  // device address of `scratch` on this device
  uint64_t launches = 0;              // calls since the status words were last cleared
};
std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

utfx_status noalloc_u8u16(const uint8_t* in, uint64_t n, uint16_t* out, uint64_t cap, void* d_result,
                          hipStream_t stream) {
  if (!d_result || (n > 0 && !in) || (cap > 0 && !out) || (reinterpret_cast<uintptr_t>(out) & 1))
    return UTFX_E_INVALID_ARG;
  if (n > UTFX_NOALLOC_MAX_BYTES) return UTFX_E_INVALID_ARG;
  if (n == 0) {
    hipLaunchKernelGGL(k_store_result, dim3(1), dim3(64), 0, stream, reinterpret_cast<Result*>(d_result), UTFX_OK,
                       0ull, 0ull);
    return hipGetLastError() == hipSuccess ? UTFX_OK : UTFX_E_DEVICE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return UTFX_E_DEVICE;
  unsigned long long* words = nullptr;
  bool clear = false;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocDevice& d = g_noalloc[dev];
    if (!d.ptr) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return UTFX_E_DEVICE;
      d.ptr = static_cast<unsigned long long*>(p);
      d.launches = 0;
    }
    // the first call on a device, and every kEpochClearEvery calls, clears the status
    // words before the 25-bit launch epoch can come round again
    clear = (d.launches % kEpochClearEvery) == 0;
    d.launches++;
    words = d.ptr;
  }
  if (clear) {
    hipLaunchKernelGGL(k_noalloc_clear, dim3(256), dim3(256), 0, stream, words, kNoAllocWords);
    if (hipGetLastError() != hipSuccess) return UTFX_E_DEVICE;
  }
  Launch L;
  const uintptr_t a = reinterpret_cast<uintptr_t>(in);
  L.base = reinterpret_cast<const uint8_t*>(a & ~static_cast<uintptr_t>(15));
  L.mis = a & 15;
  L.n = n;
  L.out = out;
  L.cap = cap;
  L.ws = reinterpret_cast<WsHeader*>(words);
  L.err = &L.ws->err;
  L.status = words + sizeof(WsHeader) / 8;
  L.result = d_result;
  L.seg = kNoAllocSeg;
  L.wg = kNoAllocWg;
  L.be = 0;
  L.dbg = 0;
  L.seg_units = kNoAllocSegUnits;
  L.ntiles = (L.mis + n + 1 + kNoAllocSegUnits - 1) / kNoAllocSegUnits;  // + 1: the position after the input
  if (L.ntiles > kNoAllocSegs) return UTFX_E_INVALID_ARG;
  hipLaunchKernelGGL((k_u8_to_u16<kNoAllocWg, kNoAllocSeg>), dim3((uint32_t)L.ntiles), dim3(kNoAllocWg), 0, stream,
                     L);
  if (hipGetLastError() != hipSuccess) return UTFX_E_DEVICE;
  hipLaunchKernelGGL(k_fin_u8u16<kNoAllocWg>, dim3(1), dim3(kNoAllocWg), 0, stream, L);
  return hipGetLastError() == hipSuccess ? UTFX_OK : UTFX_E_DEVICE;
}

}  // namespace

extern "C" {

utfx_result utfx_validate_utf32le(utfx_ctx* c, const uint32_t* in, size_t n) {
  return run_sync(c, VAL32, in, n, nullptr, 0);
}
utfx_result utfx_utf8_to_utf32le(utfx_ctx* c, const uint8_t* in, size_t n, uint32_t* out, size_t cap) {
  return run_sync(c, U8U32, in, n, out, cap);
}
utfx_result utfx_utf32le_to_utf8(utfx_ctx* c, const uint32_t* in, size_t n, uint8_t* out, size_t cap) {
  return run_sync(c, U32U8, in, n, out, cap);
}
utfx_status utfx_validate_utf32le_async(utfx_ctx* c, const uint32_t* in, size_t n, utfx_result* d_result) {
  return run(c, VAL32, in, n, nullptr, 0, d_result);
}
utfx_status utfx_utf8_to_utf32le_async(utfx_ctx* c, const uint8_t* in, size_t n, uint32_t* out, size_t cap,
                                       utfx_result* d_result) {
  return run(c, U8U32, in, n, out, cap, d_result);
}
utfx_status utfx_utf32le_to_utf8_async(utfx_ctx* c, const uint32_t* in, size_t n, uint8_t* out, size_t cap,
                                       utfx_result* d_result) {
  return run(c, U32U8, in, n, out, cap, d_result);
}

utfx_result utfx_utf16le_to_utf32le(utfx_ctx* c, const uint16_t* in, size_t n, uint32_t* out, size_t cap) {
  return run_sync(c, U16U32, in, n, out, cap);
}
utfx_result utfx_utf32le_to_utf16le(utfx_ctx* c, const uint32_t* in, size_t n, uint16_t* out, size_t cap) {
  return run_sync(c, U32U16, in, n, out, cap);
}
utfx_status utfx_utf16le_to_utf32le_async(utfx_ctx* c, const uint16_t* in, size_t n, uint32_t* out, size_t cap,
                                          utfx_result* d_result) {
  return run(c, U16U32, in, n, out, cap, d_result);
}
utfx_status utfx_utf32le_to_utf16le_async(utfx_ctx* c, const uint32_t* in, size_t n, uint16_t* out, size_t cap,
                                          utfx_result* d_result) {
  return run(c, U32U16, in, n, out, cap, d_result);
}

utfx_result utfx_utf16be_to_utf32le(utfx_ctx* c, const uint16_t* in, size_t n, uint32_t* out, size_t cap) {
  return run_sync(c, U16U32, in, n, out, cap, true);
}
utfx_result utfx_utf32le_to_utf16be(utfx_ctx* c, const uint32_t* in, size_t n, uint16_t* out, size_t cap) {
  return run_sync(c, U32U16, in, n, out, cap, true);
}
utfx_status utfx_utf16be_to_utf32le_async(utfx_ctx* c, const uint16_t* in, size_t n, uint32_t* out, size_t cap,
                                          utfx_result* d_result) {
  return run(c, U16U32, in, n, out, cap, d_result, true);
}
utfx_status utfx_utf32le_to_utf16be_async(utfx_ctx* c, const uint32_t* in, size_t n, uint16_t* out, size_t cap,
                                          utfx_result* d_result) {
  return run(c, U32U16, in, n, out, cap, d_result, true);
}

utfx_status utfx_stream_init(utfx_stream* st, int format) {
  if (!st || format < UTFX_STREAM_UTF8_TO_UTF16LE || format > UTFX_STREAM_UTF16BE_TO_UTF8)
    return UTFX_E_INVALID_ARG;
  memset(st, 0, sizeof(*st));
  st->format = format;
  st->status = UTFX_OK;
  return UTFX_OK;
}

utfx_result utfx_stream_transcode(utfx_ctx* c, utfx_stream* st, const void* in, size_t n, void* out, size_t cap,
                                  int final) {
  return stream_transcode(c, st, in, n, out, cap, final != 0);
}

utfx_status utfx_create(utfx_ctx** out, void* hip_stream) {
  if (!out) return UTFX_E_INVALID_ARG;
  *out = nullptr;
  utfx_ctx* c = new (std::nothrow) utfx_ctx();
  if (!c) return UTFX_E_DEVICE;
  c->err[0] = 0;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  // debug mode: a nonzero UTFX_DEBUG_LOOKBACK_DELAY (1..64) makes the kernels hold back
  // some segments' look-back publications (debug_delay); results must not change
  if (const char* dd = getenv("UTFX_DEBUG_LOOKBACK_DELAY")) {
    const long v = strtol(dd, nullptr, 10);
    c->dbg = v < 0 ? 0u : (v > 64 ? 64u : (uint32_t)v);
  }
  for (int i = 0; i < UTFX_OP_COUNT_; ++i) {
    c->tile_bytes[i] = 8192;
    c->seg_tiles[i] = 8;
    c->wgs_per_cu[i] = 0;
  }
  c->tile_bytes[UTFX_OP_UTF8_TO_UTF16] = 8192;
  c->seg_tiles[UTFX_OP_UTF8_TO_UTF16] = 4;
  c->tile_bytes[UTFX_OP_UTF16_TO_UTF8] = 8192;
  c->seg_tiles[UTFX_OP_UTF16_TO_UTF8] = 4;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
      c->num_cus = cus;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) == hipSuccess &&
        lds > 0)
      c->cu_lds = (uint32_t)lds;
  }
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->d_result), sizeof(Result));
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c->h_result), sizeof(Result), hipHostMallocDefault);
  if (e == hipSuccess && hipHostGetDevicePointer(reinterpret_cast<void**>(&c->h_result_dev), c->h_result, 0) != hipSuccess)
    c->h_result_dev = nullptr;
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->d_stream), sizeof(StreamDev));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&c->h_stream), sizeof(StreamRec), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&c->h_stream_dev), c->h_stream, 0);
  if (e != hipSuccess) {
    utfx_destroy(c);
    return UTFX_E_DEVICE;
  }
  if (alloc_ws(c, kInitialTiles) != UTFX_OK || batch_ws_init(c->batch) != hipSuccess) {
    utfx_destroy(c);
    return UTFX_E_DEVICE;
  }
  *out = c;
  return UTFX_OK;
}

void utfx_destroy(utfx_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  batch_ws_free(c->batch);
  if (c->ws) (void)hipFree(c->ws);
  if (c->d_result) (void)hipFree(c->d_result);
  if (c->h_result) (void)hipHostFree(c->h_result);
  if (c->d_stream) (void)hipFree(c->d_stream);
  if (c->h_stream) (void)hipHostFree(c->h_stream);
  delete c;
}

const char* utfx_last_error(const utfx_ctx* c) { return c ? c->err : "null context"; }

utfx_status utfx_set_kernel_events(utfx_ctx* c, void* start_event, void* stop_event) {
  if (!c || (!start_event) != (!stop_event)) return UTFX_E_INVALID_ARG;
  c->kev_start = reinterpret_cast<hipEvent_t>(start_event);
  c->kev_stop = reinterpret_cast<hipEvent_t>(stop_event);
  return UTFX_OK;
}

utfx_status utfx_set_stream(utfx_ctx* c, void* hip_stream) {
  if (!c) return UTFX_E_INVALID_ARG;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return UTFX_OK;
}

utfx_status utfx_set_tuning(utfx_ctx* c, int op, uint32_t tile_bytes, uint32_t tiles_per_segment,
                            uint32_t wgs_per_cu) {
  if (!c || op < 0 || op >= UTFX_OP_COUNT_ || !valid_tile(tile_bytes) || tiles_per_segment < 1 ||
      tiles_per_segment > 256 || wgs_per_cu > 16 ||
      !transcode_config_ok(op, tile_bytes, tiles_per_segment))
    return UTFX_E_INVALID_ARG;
  c->tile_bytes[op] = tile_bytes;
  c->seg_tiles[op] = tiles_per_segment;
  c->wgs_per_cu[op] = wgs_per_cu;
  return UTFX_OK;
}

utfx_status utfx_set_batch_tuning(utfx_ctx* c, uint32_t wave_max_units, uint32_t large_tiles_per_segment,
                                  uint32_t large_wgs_per_cu) {
  // the wave walkers keep positions and output offsets in 32 bits, which this upper
  // bound on the strings they take keeps far below 2^31
  if (!c || wave_max_units < 1024 || wave_max_units > (1u << 18) ||
      (large_tiles_per_segment != 2 && large_tiles_per_segment != 4) || large_wgs_per_cu < 1 || large_wgs_per_cu > 2)
    return UTFX_E_INVALID_ARG;
  c->batch_tuning.small_max = wave_max_units;
  c->batch_tuning.bs = large_tiles_per_segment;
  c->batch_tuning.large_wgs = large_wgs_per_cu;
  return UTFX_OK;
}

utfx_status utfx_get_batch_tuning(const utfx_ctx* c, uint32_t* wave_max_units, uint32_t* large_tiles_per_segment,
                                  uint32_t* large_wgs_per_cu) {
  if (!c) return UTFX_E_INVALID_ARG;
  if (wave_max_units) *wave_max_units = (uint32_t)c->batch_tuning.small_max;
  if (large_tiles_per_segment) *large_tiles_per_segment = c->batch_tuning.bs;
  if (large_wgs_per_cu) *large_wgs_per_cu = c->batch_tuning.large_wgs;
  return UTFX_OK;
}

utfx_status utfx_get_tuning(const utfx_ctx* c, int op, uint32_t* tile_bytes, uint32_t* tiles_per_segment,
                            uint32_t* wgs_per_cu) {
  if (!c || op < 0 || op >= UTFX_OP_COUNT_) return UTFX_E_INVALID_ARG;
  if (tile_bytes) *tile_bytes = c->tile_bytes[op];
  if (tiles_per_segment) *tiles_per_segment = c->seg_tiles[op];
  if (wgs_per_cu) *wgs_per_cu = c->wgs_per_cu[op];
  return UTFX_OK;
}

utfx_result utfx_utf16_length_from_utf8(utfx_ctx* c, const uint8_t* in, size_t n) {
  return run_sync(c, LEN8, in, n, nullptr, 0);
}
utfx_result utfx_utf8_length_from_utf16le(utfx_ctx* c, const uint16_t* in, size_t n) {
  return run_sync(c, LEN16, in, n, nullptr, 0);
}
utfx_result utfx_validate_utf8(utfx_ctx* c, const uint8_t* in, size_t n) {
  return run_sync(c, VAL8, in, n, nullptr, 0);
}
utfx_result utfx_validate_utf16le(utfx_ctx* c, const uint16_t* in, size_t n) {
  return run_sync(c, VAL16, in, n, nullptr, 0);
}
utfx_result utfx_utf8_to_utf16le(utfx_ctx* c, const uint8_t* in, size_t n, uint16_t* out, size_t cap) {
  return run_sync(c, U8U16, in, n, out, cap);
}
utfx_result utfx_utf16le_to_utf8(utfx_ctx* c, const uint16_t* in, size_t n, uint8_t* out, size_t cap) {
  return run_sync(c, U16U8, in, n, out, cap);
}

utfx_status utfx_utf16_length_from_utf8_async(utfx_ctx* c, const uint8_t* in, size_t n, utfx_result* r) {
  return run(c, LEN8, in, n, nullptr, 0, r);
}
utfx_status utfx_utf8_length_from_utf16le_async(utfx_ctx* c, const uint16_t* in, size_t n, utfx_result* r) {
  return run(c, LEN16, in, n, nullptr, 0, r);
}
utfx_status utfx_validate_utf8_async(utfx_ctx* c, const uint8_t* in, size_t n, utfx_result* r) {
  return run(c, VAL8, in, n, nullptr, 0, r);
}
utfx_status utfx_validate_utf16le_async(utfx_ctx* c, const uint16_t* in, size_t n, utfx_result* r) {
  return run(c, VAL16, in, n, nullptr, 0, r);
}
utfx_status utfx_utf8_to_utf16le_async(utfx_ctx* c, const uint8_t* in, size_t n, uint16_t* out, size_t cap,
                                       utfx_result* r) {
  return run(c, U8U16, in, n, out, cap, r);
}
utfx_status utfx_utf16le_to_utf8_async(utfx_ctx* c, const uint16_t* in, size_t n, uint8_t* out, size_t cap,
                                       utfx_result* r) {
  return run(c, U16U8, in, n, out, cap, r);
}

utfx_status utfx_utf8_to_utf16le_noalloc(const uint8_t* in, size_t n, uint16_t* out, size_t cap, utfx_result* r,
                                         void* hip_stream) {
  return noalloc_u8u16(in, n, out, cap, r, reinterpret_cast<hipStream_t>(hip_stream));
}

utfx_result utfx_utf8_length_from_utf16be(utfx_ctx* c, const uint16_t* in, size_t n) {
  return run_sync(c, LEN16, in, n, nullptr, 0, true);
}
utfx_result utfx_validate_utf16be(utfx_ctx* c, const uint16_t* in, size_t n) {
  return run_sync(c, VAL16, in, n, nullptr, 0, true);
}
utfx_result utfx_utf8_to_utf16be(utfx_ctx* c, const uint8_t* in, size_t n, uint16_t* out, size_t cap) {
  return run_sync(c, U8U16, in, n, out, cap, true);
}
utfx_result utfx_utf16be_to_utf8(utfx_ctx* c, const uint16_t* in, size_t n, uint8_t* out, size_t cap) {
  return run_sync(c, U16U8, in, n, out, cap, true);
}
utfx_status utfx_utf8_length_from_utf16be_async(utfx_ctx* c, const uint16_t* in, size_t n, utfx_result* r) {
  return run(c, LEN16, in, n, nullptr, 0, r, true);
}
utfx_status utfx_validate_utf16be_async(utfx_ctx* c, const uint16_t* in, size_t n, utfx_result* r) {
  return run(c, VAL16, in, n, nullptr, 0, r, true);
}
utfx_status utfx_utf8_to_utf16be_async(utfx_ctx* c, const uint8_t* in, size_t n, uint16_t* out, size_t cap,
                                       utfx_result* r) {
  return run(c, U8U16, in, n, out, cap, r, true);
}
utfx_status utfx_utf16be_to_utf8_async(utfx_ctx* c, const uint16_t* in, size_t n, uint8_t* out, size_t cap,
                                       utfx_result* r) {
  return run(c, U16U8, in, n, out, cap, r, true);
}

utfx_status utfx_batch_run(utfx_ctx* c, const uint8_t* in_arena, size_t in_bytes, uint8_t* out_arena,
                           size_t out_bytes, const utfx_item* d_items, uint32_t n_items, uint64_t total_in_units,
                           utfx_result* d_results) {
  if (!c) return UTFX_E_INVALID_ARG;
  c->err[0] = 0;
  const uint64_t gen = c->batch.gen;
  utfx_status st = batch_run(c->batch, c->stream, c->capturing, c->num_cus, c->dbg, c->batch_tuning, in_arena,
                             in_bytes, out_arena, out_bytes, d_items, n_items, total_in_units, d_results, c->err,
                             sizeof(c->err));
  if (c->batch.gen != gen) c->ws_gen++;  // kernels captured before hold freed addresses
  if (st == UTFX_OK && c->capturing) c->cap_batches++;
  return st;
}

utfx_status utfx_capture_begin(utfx_ctx* c) {
  if (!c || c->capturing) return UTFX_E_INVALID_ARG;
  c->err[0] = 0;
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    set_err(c, "begin capture", e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    return UTFX_E_DEVICE;
  }
  c->user_stream = c->stream;
  c->stream = c->cap_stream;
  c->capturing = true;
  c->cap_launches = 0;
  c->cap_batches = 0;
  return UTFX_OK;
}

utfx_status utfx_capture_end(utfx_ctx* c, utfx_graph** out) {
  if (!c || !c->capturing || !out) return UTFX_E_INVALID_ARG;
  *out = nullptr;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  c->stream = c->user_stream;
  c->capturing = false;
  (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  if (e != hipSuccess || !graph) {
    set_err(c, "end capture", e);
    return UTFX_E_DEVICE;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    set_err(c, "instantiate graph", e);
    (void)hipGraphDestroy(graph);
    return UTFX_E_DEVICE;
  }
  utfx_graph* g = new (std::nothrow) utfx_graph();
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return UTFX_E_DEVICE;
  }
  g->ctx = c;
  g->graph = graph;
  g->exec = exec;
  g->launches = c->cap_launches;
  g->batches = c->cap_batches;
  g->ws_gen = c->ws_gen;
  *out = g;
  return UTFX_OK;
}

utfx_status utfx_graph_launch(utfx_graph* g, void* hip_stream) {
  if (!g || g->ctx->capturing) return UTFX_E_INVALID_ARG;
  utfx_ctx* c = g->ctx;
  if (g->ws_gen != c->ws_gen) {
    // the graph's kernels hold the addresses of a workspace that has since been freed
    set_msg(c, "the context's workspace grew after this graph was captured; capture it again");
    return UTFX_E_INVALID_ARG;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  // replays advance the workspace epochs like eager calls; clear the status words
  // before the epoch space could wrap
  if (c->launches + g->launches >= kEpochClearEvery) {
    (void)hipStreamSynchronize(s);
    if (init_ws(c) != UTFX_OK) return UTFX_E_DEVICE;
  }
  if (c->batch.launches + g->batches >= (1ull << 24)) {
    (void)hipStreamSynchronize(s);
    if (batch_ws_clear(c->batch, c->stream) != hipSuccess) return UTFX_E_DEVICE;
  }
  hipError_t e = hipGraphLaunch(g->exec, s);
  if (e != hipSuccess) {
    set_err(c, "graph launch", e);
    return UTFX_E_DEVICE;
  }
  c->launches += g->launches;
  c->batch.launches += g->batches;
  return UTFX_OK;
}

void utfx_graph_destroy(utfx_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"

#include "utfx_serve.hpp"
