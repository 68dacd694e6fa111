// Host side of the C ABI declared in include/mi355scan.h: argument checks,
// per-stream workspaces, configuration dispatch, launches, graphs and the
// autotuner.  Every step of the scan itself runs in the HIP kernels of
// scan_kernels.hip; this file only prepares launches.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mi355scan.h"
#include "scan_shared.hpp"
#include "scan_table.hpp"
#include "validate.hpp"

// Workspace of scan_flat_noalloc, the entry point for callers that cannot
// allocate: a library array in device memory (one copy per device, zero at
// module load, held until the process ends) laid out as a stream workspace
// without tile map and two-pass sums: header | publish counters |
// status[2][kScratchTiles].  The kernels raise the header's `error` word on a
// timeout.  In host code `scratch` only names the symbol: its device address
// comes from hipGetSymbolAddress (per device, see scratch_ws).
namespace mi355scan {
constexpr int64_t kScratchTiles = int64_t(1) << 15;
constexpr size_t kScratchBytes =
    sizeof(WsHeader) + kPubWords * sizeof(uint64_t) + (size_t)kScratchTiles * 2 * sizeof(uint64_t);
static_assert(kScratchBytes % sizeof(uint64_t) == 0, "scratch layout");
}  // namespace mi355scan
static __device__ __align__(256) uint64_t scratch[mi355scan::kScratchBytes / sizeof(uint64_t)];

namespace mi355scan {
namespace {

// A legitimate wait never outlasts the whole kernel (about a millisecond at
// 2^30 elements); 2^16 sleeping polls is of the order of 0.1 s.
constexpr uint32_t kDefaultSpinLimit = 1u << 16;
constexpr int kDefaultFlatConfig = 22;  // 768 threads x 128 items, one resident workgroup per CU
constexpr int kDefaultSegConfig = 20;   // 512 threads x 128 items, one resident workgroup per CU
// The autotuner takes a configuration whose tile order relies on the
// dispatcher (mode 2: tile = workgroup index, in-order dispatch assumed) or
// on co-residency (mode 4) only when it beats the best counter-mode
// configuration by more than this fraction; otherwise timing noise would
// decide between them.
constexpr float kOrderedMargin = 0.03f;
constexpr int kBuckets = 64;

thread_local int t_last_hip = 0;
std::mutex g_mu;
uint32_t g_spin_limit = kDefaultSpinLimit;
int g_forced = -1;
int g_table[2][2][kBuckets];      // [int / f32][segmented][floor(log2 n)] -> config, -1 = default

scan_status_t st(int s) { return static_cast<scan_status_t>(s); }

scan_status_t hip_fail(hipError_t e, scan_status_t code = SCAN_ERROR_LAUNCH) {
  t_last_hip = (int)e;
  return code;
}

int bucket_of(int64_t n) {
  int b = 0;
  while (b < kBuckets - 1 && (int64_t(1) << (b + 1)) <= n) ++b;
  return b;
}

int opclass_of(scan_dtype_t dt) { return dt == SCAN_F32 ? 1 : 0; }

// ------------------------------------------------------------------ devices
struct DeviceInfo {
  bool supported = false;
  int cus = 0;
};
std::map<int, DeviceInfo> g_devices;

scan_status_t current_device(int *dev, DeviceInfo *info) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, SCAN_ERROR_NOT_SUPPORTED);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_devices.find(*dev);
  if (it == g_devices.end()) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, *dev);
    if (e != hipSuccess) return hip_fail(e, SCAN_ERROR_NOT_SUPPORTED);
    DeviceInfo di;
    di.supported = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    di.cus = prop.multiProcessorCount;
    it = g_devices.emplace(*dev, di).first;
  }
  *info = it->second;
  return info->supported ? SCAN_SUCCESS : SCAN_ERROR_NOT_SUPPORTED;
}

// --------------------------------------------------------------- workspaces
// Layout of one allocation: header (64 B) | publish counters (kPubWords u64) |
// status[2][capacity] (u64) | tile map[capacity + 1] (u32).
struct Workspace {
  int device = -1;
  char *base = nullptr;
  WsHeader *hdr = nullptr;
  uint64_t *pubcnt = nullptr;
  uint64_t *status = nullptr;
  uint32_t *map = nullptr;
  uint64_t *sums = nullptr;   // two-pass scans: capacity tile totals + one running total
  uint32_t *err = nullptr;    // error word the kernels raise on a timeout (device view)
  int64_t capacity = 0;   // tiles
};

// A word of pinned, coherent host memory that kernels raise (system-scope
// store) when a wait gives up: the host reads it without synchronising.
scan_status_t err_alloc(uint32_t **host, uint32_t **dev) {
  void *p = nullptr;
  hipError_t e = hipHostMalloc(&p, 64, hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return hip_fail(e, SCAN_ERROR_OUT_OF_MEMORY);
  void *d = nullptr;
  e = hipHostGetDevicePointer(&d, p, 0);
  if (e != hipSuccess) {
    (void)hipHostFree(p);
    return hip_fail(e);
  }
  __atomic_store_n(static_cast<uint32_t *>(p), 0u, __ATOMIC_RELEASE);
  *host = static_cast<uint32_t *>(p);
  *dev = static_cast<uint32_t *>(d);
  return SCAN_SUCCESS;
}

void err_free(uint32_t **host, uint32_t **dev) {
  if (*host) (void)hipHostFree(*host);
  *host = nullptr;
  *dev = nullptr;
}

// Read and clear an error word: true if a wait gave up since the last read.
bool take_error(uint32_t *host) {
  return host && __atomic_exchange_n(host, 0u, __ATOMIC_ACQ_REL) != 0u;
}

constexpr size_t kStatusOffset = sizeof(WsHeader) + kPubWords * sizeof(uint64_t);

size_t map_offset(int64_t cap) { return kStatusOffset + (size_t)cap * 2 * sizeof(uint64_t); }
size_t sums_offset(int64_t cap) {
  return (map_offset(cap) + (size_t)(cap + 1) * sizeof(uint32_t) + 7) & ~(size_t)7;
}
size_t ws_bytes(int64_t cap) { return sums_offset(cap) + (size_t)(cap + 1) * sizeof(uint64_t); }

scan_status_t ws_alloc(Workspace *w, int device, int64_t cap, hipStream_t stream) {
  const size_t bytes = ws_bytes(cap);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return hip_fail(e, SCAN_ERROR_OUT_OF_MEMORY);
  e = hipMemsetAsync(p, 0, bytes, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_fail(e);
  }
  w->device = device;
  w->base = static_cast<char *>(p);
  w->hdr = reinterpret_cast<WsHeader *>(w->base);
  w->pubcnt = reinterpret_cast<uint64_t *>(w->base + sizeof(WsHeader));
  w->status = reinterpret_cast<uint64_t *>(w->base + kStatusOffset);
  w->map = reinterpret_cast<uint32_t *>(w->base + map_offset(cap));
  w->sums = reinterpret_cast<uint64_t *>(w->base + sums_offset(cap));
  w->capacity = cap;
  return SCAN_SUCCESS;
}

void ws_free(Workspace *w) {
  if (w->base) (void)hipFree(w->base);
  *w = Workspace();
}

// Per (device, stream): the current workspace, the allocations it outgrew
// (kept until scan_release: graphs captured from this stream's calls still
// use them) and the stream's error word, shared by all of them.
struct StreamState {
  Workspace ws;
  std::vector<Workspace> retired;
  uint32_t *err_host = nullptr;
  uint32_t *err_dev = nullptr;
};
std::map<std::pair<int, hipStream_t>, StreamState> g_ws;

// The allocation-free workspace of each device: the device address of that
// device's copy of `scratch`, taken once with the device current.
std::map<int, Workspace> g_scratch;

scan_status_t scratch_ws(int device, Workspace **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end()) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e);
    Workspace w;
    w.device = device;
    w.base = static_cast<char *>(p);
    w.hdr = reinterpret_cast<WsHeader *>(w.base);
    w.pubcnt = reinterpret_cast<uint64_t *>(w.base + sizeof(WsHeader));
    w.status = reinterpret_cast<uint64_t *>(w.base + kStatusOffset);
    w.err = &w.hdr->error;
    w.capacity = kScratchTiles;
    it = g_scratch.emplace(device, w).first;
  }
  *out = &it->second;
  return SCAN_SUCCESS;
}

// The scratch workspace of `device` if a call has set it up, else null.
Workspace *scratch_ws_if_set(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(device);
  return it == g_scratch.end() ? nullptr : &it->second;
}

// A timeout raised by an earlier launch on this stream is reported (once) by
// the next call, which then enqueues nothing: its results could not be told
// apart from those of the call that failed.
scan_status_t stream_pending(int device, hipStream_t stream) {
  uint32_t *h = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find(std::make_pair(device, stream));
    if (it != g_ws.end()) h = it->second.err_host;
  }
  return take_error(h) ? SCAN_ERROR_TIMEOUT : SCAN_SUCCESS;
}

int64_t min_tile() {
  int64_t m = (int64_t)kUnalignedShape.block * kUnalignedShape.items;
  for (int i = 0; i < kNumShapes; ++i) m = std::min<int64_t>(m, (int64_t)kShapes[i].block * kShapes[i].items);
  return m;
}

int64_t tiles_for(int64_t n, int64_t tile) { return (n + tile - 1) / tile; }

// The stream's workspace with room for `need` tiles.  Growing allocates a
// new one and retires the old one without freeing it: a graph the caller
// captured from this stream's calls keeps using the old allocation, which
// stays valid and clean until scan_release.
scan_status_t stream_ws(int device, hipStream_t stream, int64_t need, Workspace **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  StreamState &ss = g_ws[std::make_pair(device, stream)];
  if (ss.ws.base && ss.ws.capacity >= need) {
    *out = &ss.ws;
    return SCAN_SUCCESS;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(stream, &cs);
  if (e != hipSuccess) return hip_fail(e);
  if (cs != hipStreamCaptureStatusNone) return SCAN_ERROR_CAPTURE;
  if (!ss.err_host) {
    scan_status_t s = err_alloc(&ss.err_host, &ss.err_dev);
    if (s != SCAN_SUCCESS) return s;
  }
  const int64_t cap = std::max<int64_t>({need, 2 * ss.ws.capacity, 1024});
  Workspace nw;
  scan_status_t s = ws_alloc(&nw, device, cap, stream);
  if (s != SCAN_SUCCESS) return s;
  nw.err = ss.err_dev;
  if (ss.ws.base) ss.retired.push_back(ss.ws);
  ss.ws = nw;
  *out = &ss.ws;
  return SCAN_SUCCESS;
}

// ---------------------------------------------------------------- tuning
void load_default_tune_file();

std::once_flag g_init_once;

void ensure_init() {
  std::call_once(g_init_once, [] {
    {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto &a : g_table)
        for (auto &b : a)
          for (int &c : b) c = -1;
    }
    load_default_tune_file();
  });
}

int select_config(int opclass, bool seg, int64_t n) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_forced >= 0) return g_forced;
  const int c = g_table[opclass][seg ? 1 : 0][bucket_of(n)];
  if (c >= 0 && c < kNumConfigs) return c;
  return seg ? kDefaultSegConfig : kDefaultFlatConfig;
}

std::map<const void *, int> g_occupancy;

int resident_blocks(const void *fn, int block, int cus) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_occupancy.find(fn);
    if (it != g_occupancy.end()) return it->second * cus;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  std::lock_guard<std::mutex> lk(g_mu);
  g_occupancy[fn] = per_cu;
  return per_cu * cus;
}

// Workgroups of a resident grid: per_cu per CU when given (never more than
// fit), else as many as fit, on cu_pct percent of the CUs.
int64_t resident_grid(const void *fn, int block, int cus, int per_cu, int cu_pct) {
  const int64_t fit = resident_blocks(fn, block, cus);
  const int64_t want = per_cu > 0 ? std::min<int64_t>(fit, (int64_t)per_cu * cus) : fit;
  return std::max<int64_t>(1, want * cu_pct / 100);
}

// ---------------------------------------------------------------- launching
struct Call {
  const void *in;
  void *out;
  int64_t n;
  int opclass;   // tuning class: 0 = 32-bit integer, 1 = float32
  bool seg;
  uint32_t flags;
  const int64_t *offsets;
  int64_t num_segments;
  int kind = 0;        // kernel kind (operator), see kernel_kind
  uint32_t key = 0u;   // keyed max: x ^ key
};

Call make_call(const void *in, void *out, int64_t n, scan_dtype_t dt, bool seg, uint32_t flags,
               const int64_t *offsets, int64_t num_segments) {
  Call c{in, out, n, opclass_of(dt), seg, flags, offsets, num_segments};
  c.kind = kernel_kind((int)dt, flags);
  c.key = op_key((int)dt, flags);
  return c;
}

bool call_aligned(const Call &c) {
  return ((uintptr_t)c.in & 15u) == 0 && ((uintptr_t)c.out & 15u) == 0;
}

// Kernel shape and tile mode a call runs with under configuration cfg:
// buffers that are not 16-byte aligned take the dword-access kernels with a
// resident grid.
const KernelShape &call_shape(const Call &c, int cfg) {
  return call_aligned(c) ? kShapes[kConfigs[cfg].shape] : kUnalignedShape;
}
int call_mode(const Call &c, int cfg) { return call_aligned(c) ? kConfigs[cfg].mode : (int)kModePersistent; }
int call_per_cu(const Call &c, int cfg) { return call_aligned(c) ? kConfigs[cfg].per_cu : 0; }
int call_cu_pct(const Call &c, int cfg) { return call_aligned(c) ? kConfigs[cfg].cu_pct : 100; }

// Tiles a call of this shape needs under configuration cfg.
int64_t call_tiles(const Call &c, int cfg) {
  const KernelShape &sh = call_shape(c, cfg);
  return tiles_for(c.n, (int64_t)sh.block * sh.items);
}

// Tile indices (and byte offsets into a status array) must fit in 32 bits.
constexpr int64_t kMaxTiles = int64_t(1) << 29;

// Enqueue one scan (plus the tile map for segmented calls).  ws_override is a
// graph-owned workspace (already large enough) or null for the stream's own.
scan_status_t launch(const Call &c, hipStream_t stream, Workspace *ws_override, int cfg_override) {
  if (c.n == 0) return SCAN_SUCCESS;
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  if (!ws_override) {
    s = stream_pending(dev, stream);
    if (s != SCAN_SUCCESS) return s;
  }
  const int cfg = cfg_override >= 0 ? cfg_override : select_config(c.opclass, c.seg, c.n);
  const KernelShape &sh = call_shape(c, cfg);
  const int mode = call_mode(c, cfg);
  const int64_t tile = (int64_t)sh.block * sh.items;
  const int64_t T = tiles_for(c.n, tile);
  if (T > kMaxTiles) return SCAN_ERROR_NOT_SUPPORTED;
  const int per_cu = call_per_cu(c, cfg);
  const void *fn = sh.fn[c.kind][c.seg ? 1 : 0][(c.flags & SCAN_REVERSE) ? 1 : 0];
  const int cu_pct = call_cu_pct(c, cfg);

  Workspace *ws = nullptr;
  if (T > 1) {
    if (ws_override) {
      if (ws_override->capacity < T) return SCAN_ERROR_INVALID_VALUE;
      ws = ws_override;
    } else {
      s = stream_ws(dev, stream, T, &ws);
      if (s != SCAN_SUCCESS) return s;
    }
  }

  KernelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = c.in;
  a.out = c.out;
  a.n = c.n;
  a.tiles = T;
  a.hdr = ws ? ws->hdr : nullptr;
  a.status = ws ? ws->status : nullptr;
  a.capacity = ws ? ws->capacity : 0;
  a.offsets = c.offsets;
  a.tile_seg = nullptr;
  a.num_segments = c.num_segments;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    a.spin_limit = g_spin_limit;
  }
  a.err = ws ? ws->err : nullptr;
  a.exclusive = (c.flags & SCAN_EXCLUSIVE) ? 1u : 0u;
  a.reverse = (c.flags & SCAN_REVERSE) ? 1u : 0u;
  a.key = c.key;

  const int threads = sh.block;
  int64_t grid = T;
  a.one_tile = 1u;
  a.ordered = 0u;
  a.pubcnt = ws ? ws->pubcnt : nullptr;
  bool cooperative = false;
  if (T > 1 && mode == kModeOrdered) {
    a.ordered = 1u;
    a.total_acquires = 0;
  } else if (T > 1 && mode == kModeStatic) {
    grid = std::min<int64_t>(T, resident_grid(fn, threads, di.cus, per_cu, cu_pct));
    a.one_tile = 0u;
    a.stride = (uint32_t)grid;
    a.total_acquires = 0;
    cooperative = true;
  } else if (T > 1 && mode == kModePersistent) {
    grid = std::min<int64_t>(T, resident_grid(fn, threads, di.cus, per_cu, cu_pct));
    a.one_tile = grid == T ? 1u : 0u;
    a.total_acquires = a.one_tile ? (uint64_t)T : (uint64_t)(T + grid);
  } else {
    a.total_acquires = (uint64_t)T;
  }
  if (c.seg && T > 1) {
    const int64_t cnt = T + 1;
    const int mb = 256;
    const int64_t mgrid = (cnt + mb - 1) / mb;
    const int64_t *off = c.offsets;
    int64_t S = c.num_segments;
    int64_t tl = tile;
    int32_t shift = a.reverse ? 1 : 0;
    uint32_t *map = ws->map;
    void *margs[] = {&off, &S, &tl, (void *)&T, &shift, &map};
    hipError_t e = hipLaunchKernel(kTileSegmentMap, dim3((unsigned)mgrid), dim3(mb), margs, 0, stream);
    if (e != hipSuccess) return hip_fail(e);
    a.tile_seg = ws->map;
  }
  void *kargs[] = {&a};
  // a cooperative launch guarantees that the whole grid is resident at once,
  // which the static round robin needs for forward progress
  hipError_t e = cooperative
                     ? hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(threads), kargs, 0, stream)
                     : hipLaunchKernel(fn, dim3((unsigned)grid), dim3(threads), kargs, 0, stream);
  if (e != hipSuccess) return hip_fail(e);
  return SCAN_SUCCESS;
}

// 64-bit scans: one resident launch of the 64-bit kernel over 32768-element
// tiles (tiles from the counter), two status words per tile.
scan_status_t flat64(const void *in, void *out, int64_t n, scan_dtype_t dt, uint32_t flags,
                     hipStream_t stream) {
  int r = check_flags(flags);
  if (r == kOk) r = check_flat_sz(in, out, n, 8);
  if (r != kOk) return st(r);
  if (flags & ~(uint32_t)(SCAN_EXCLUSIVE | SCAN_REVERSE)) return SCAN_ERROR_NOT_SUPPORTED;   // +-scans only
  if (((uintptr_t)in & 15u) || ((uintptr_t)out & 15u)) return SCAN_ERROR_INVALID_VALUE;
  if (n == 0) return SCAN_SUCCESS;
  ensure_init();
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  s = stream_pending(dev, stream);
  if (s != SCAN_SUCCESS) return s;
  const int kind = dt == SCAN_F64 ? 1 : 0;
  const int64_t tile = (int64_t)kScan64Block[kind] * kScan64Items[kind];
  const int64_t T = tiles_for(n, tile);
  if (2 * T > kMaxTiles) return SCAN_ERROR_NOT_SUPPORTED;
  Workspace *ws = nullptr;
  if (T > 1) {
    s = stream_ws(dev, stream, 2 * T, &ws);
    if (s != SCAN_SUCCESS) return s;
  }
  const void *fn = kScan64[kind][(flags & SCAN_REVERSE) ? 1 : 0];
  const int64_t grid = std::min<int64_t>(T, resident_grid(fn, kScan64Block[kind], di.cus, 0, 100));
  KernelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.n = n;
  a.tiles = T;
  a.hdr = ws ? ws->hdr : nullptr;
  a.status = ws ? ws->status : nullptr;
  a.capacity = ws ? ws->capacity : 0;
  a.total_acquires = (uint64_t)(T + grid);   // every workgroup also takes one tile past the end
  {
    std::lock_guard<std::mutex> lk(g_mu);
    a.spin_limit = g_spin_limit;
  }
  a.err = ws ? ws->err : nullptr;
  a.exclusive = (flags & SCAN_EXCLUSIVE) ? 1u : 0u;
  void *args[] = {&a};
  hipError_t e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kScan64Block[kind]), args, 0, stream);
  return e == hipSuccess ? SCAN_SUCCESS : hip_fail(e);
}

scan_status_t flat(const void *in, void *out, int64_t n, scan_dtype_t dt, uint32_t flags,
                   hipStream_t stream) {
  if (is_dtype64((int)dt)) return flat64(in, out, n, dt, flags, stream);
  int r = check_dtype((int)dt);
  if (r == kOk) r = check_flags(flags);
  if (r == kOk) r = check_flat(in, out, n);
  if (r == kOk) r = check_operator((int)dt, flags);
  if (r != kOk) return st(r);
  if (n == 0) return SCAN_SUCCESS;
  ensure_init();
  Call c = make_call(in, out, n, dt, false, flags, nullptr, 0);
  return launch(c, stream, nullptr, -1);
}

// The streaming-ceiling kernel (stream_ceiling.hpp) with the tile shape,
// grid and tile counter of configuration cfg (counter modes only).
scan_status_t stream_ceiling(const void *in, void *out, int64_t n, int32_t cfg, hipStream_t stream) {
  const int r = check_flat(in, out, n);
  if (r != kOk) return st(r);
  if (cfg < 0 || cfg >= kNumConfigs) return SCAN_ERROR_INVALID_VALUE;
  if (((uintptr_t)in | (uintptr_t)out) & 15u) return SCAN_ERROR_INVALID_VALUE;
  const Config &cf = kConfigs[cfg];
  if (cf.mode != kModeCounter && cf.mode != kModePersistent) return SCAN_ERROR_NOT_SUPPORTED;
  if (n == 0) return SCAN_SUCCESS;
  ensure_init();
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  s = stream_pending(dev, stream);
  if (s != SCAN_SUCCESS) return s;
  const KernelShape &sh = kShapes[cf.shape];
  const int64_t T = tiles_for(n, (int64_t)sh.block * sh.items);
  if (T > kMaxTiles) return SCAN_ERROR_NOT_SUPPORTED;
  Workspace *ws = nullptr;
  if (T > 1) {
    s = stream_ws(dev, stream, T, &ws);
    if (s != SCAN_SUCCESS) return s;
  }
  KernelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.n = n;
  a.tiles = T;
  a.hdr = ws ? ws->hdr : nullptr;
  a.status = ws ? ws->status : nullptr;
  a.capacity = ws ? ws->capacity : 0;
  a.err = ws ? ws->err : nullptr;
  int64_t grid = T;
  a.one_tile = 1u;
  a.total_acquires = (uint64_t)T;
  if (T > 1 && cf.mode != kModeCounter) {
    grid = std::min<int64_t>(T, resident_grid(sh.copy, sh.block, di.cus, cf.per_cu, cf.cu_pct));
    a.one_tile = grid == T ? 1u : 0u;
    a.total_acquires = a.one_tile ? (uint64_t)T : (uint64_t)(T + grid);
  }
  void *args[] = {&a};
  hipError_t e = hipLaunchKernel(sh.copy, dim3((unsigned)grid), dim3(sh.block), args, 0, stream);
  return e == hipSuccess ? SCAN_SUCCESS : hip_fail(e);
}

// Flat 32-bit scan on the device's scratch workspace: the tuned
// configuration when its tiles fit the scratch, else the default one (the
// largest tiles), else the call is refused.  Nothing is allocated.
scan_status_t flat_noalloc(const void *in, void *out, int64_t n, scan_dtype_t dt, uint32_t flags,
                           hipStream_t stream) {
  int r = check_dtype((int)dt);
  if (r == kOk) r = check_flags(flags);
  if (r == kOk) r = check_flat(in, out, n);
  if (r == kOk) r = check_operator((int)dt, flags);
  if (r != kOk) return st(r);
  if (n == 0) return SCAN_SUCCESS;
  ensure_init();
  Call c = make_call(in, out, n, dt, false, flags, nullptr, 0);
  int cfg = select_config(c.opclass, false, n);
  if (call_tiles(c, cfg) > kScratchTiles) cfg = kDefaultFlatConfig;
  if (call_tiles(c, cfg) > kScratchTiles) return SCAN_ERROR_INVALID_VALUE;
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  Workspace *ws = nullptr;
  s = scratch_ws(dev, &ws);
  if (s != SCAN_SUCCESS) return s;
  return launch(c, stream, ws, cfg);
}

scan_status_t segmented(const void *in, void *out, const int64_t *offsets, int32_t S, int64_t n,
                        scan_dtype_t dt, uint32_t flags, hipStream_t stream, Workspace *ws, int cfg) {
  int r = check_dtype((int)dt);
  if (r == kOk) r = check_flags(flags);
  if (r == kOk) r = check_segmented(in, out, offsets, S, n);
  if (r == kOk) r = check_operator((int)dt, flags);
  if (r != kOk) return st(r);
  if (n == 0) return SCAN_SUCCESS;
  ensure_init();
  Call c = make_call(in, out, n, dt, true, flags, offsets, S);
  return launch(c, stream, ws, cfg);
}

// Two-pass scans (Section 2.1), partition by partition (Section 2.2): per
// partition, pass 1 over its tiles, the scan of their totals (one
// workgroup, which also carries the running total of the partitions before),
// pass 2.  All launches go to `stream` in order.
scan_status_t two_pass(const void *in, void *out, int64_t n, scan_dtype_t dt, uint32_t flags,
                       int32_t method, int64_t partition, hipStream_t stream) {
  int r = check_dtype((int)dt);
  if (r == kOk) r = check_flags(flags);
  if (r == kOk) r = check_flat(in, out, n);
  if (r != kOk) return st(r);
  if (op_of(flags) != kOpSum) return SCAN_ERROR_NOT_SUPPORTED;
  if (method != SCAN_TWO_PASS_PREFIX_INCREMENT && method != SCAN_TWO_PASS_ACCUMULATE_PREFIX)
    return SCAN_ERROR_INVALID_VALUE;
  if (partition < 0) return SCAN_ERROR_INVALID_VALUE;
  if (flags & SCAN_REVERSE) return SCAN_ERROR_NOT_SUPPORTED;
  if (n == 0) return SCAN_SUCCESS;
  ensure_init();
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  s = stream_pending(dev, stream);
  if (s != SCAN_SUCCESS) return s;
  const TwoPassKernels &K = kTwoPass;
  const int64_t tile = (int64_t)K.block * K.items;
  const int64_t T = tiles_for(n, tile);
  if (T > kMaxTiles) return SCAN_ERROR_NOT_SUPPORTED;
  Workspace *ws = nullptr;
  s = stream_ws(dev, stream, T, &ws);
  if (s != SCAN_SUCCESS) return s;
  const int op = opclass_of(dt);
  const int vec = (((uintptr_t)in | (uintptr_t)out) & 15u) == 0 ? 1 : 0;
  const int64_t per = partition == 0 ? T : std::max<int64_t>(1, tiles_for(partition, tile));
  // pass 1 hands its data to pass 2 through the caches only when partitioned
  const int nt1 = per >= T ? 1 : 0;
  const bool acc = method == SCAN_TWO_PASS_ACCUMULATE_PREFIX;
  const void *pass1 = acc ? K.totals[op][vec][nt1] : K.local_scan[op][vec][nt1];
  const void *pass2 = acc ? K.offset_scan[op][vec] : K.increment[op][vec];

  TwoPassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k.in = in;
  a.k.out = out;
  a.k.n = n;
  a.k.tiles = T;
  a.k.exclusive = (flags & SCAN_EXCLUSIVE) ? 1u : 0u;
  a.sums = ws->sums;
  a.run = ws->sums + ws->capacity;
  for (int64_t t0 = 0; t0 < T; t0 += per) {
    a.tile0 = t0;
    a.ntiles = std::min<int64_t>(per, T - t0);
    void *args[] = {&a};
    hipError_t e = hipLaunchKernel(pass1, dim3((unsigned)a.ntiles), dim3(K.block), args, 0, stream);
    if (e == hipSuccess)
      e = hipLaunchKernel(K.scan_totals[op], dim3(1), dim3(K.totals_block), args, 0, stream);
    if (e == hipSuccess) e = hipLaunchKernel(pass2, dim3((unsigned)a.ntiles), dim3(K.block), args, 0, stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  return SCAN_SUCCESS;
}

// Stream compaction fused with the exclusive scan: one resident launch over
// 65536-element tiles (tiles from the counter, as the scan's mode 1).
// part: the two-way partition (rejected elements to the end, reversed), which
// writes ahead of the tiles still to be read and so cannot run in place.
scan_status_t compact(const void *in, void *out, int64_t n, scan_dtype_t dt, int32_t predicate,
                      uint32_t threshold, int64_t *count, hipStream_t stream, bool part = false) {
  int r = check_dtype((int)dt);
  if (r == kOk) r = check_flat(in, out, n);
  if (r == kOk && part && n > 0 && in == out) r = kOverlap;
  if (r != kOk) return st(r);
  if (!count || ((uintptr_t)count & 7u)) return SCAN_ERROR_INVALID_VALUE;
  if (predicate != SCAN_PRED_NONZERO && predicate != SCAN_PRED_GREATER) return SCAN_ERROR_INVALID_VALUE;
  if (n > (int64_t)0xFFFFFFFF) return SCAN_ERROR_NOT_SUPPORTED;   // counts are 32-bit
  ensure_init();
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  s = stream_pending(dev, stream);
  if (s != SCAN_SUCCESS) return s;
  // the partition kernels have their own shape; the n = 0 count kernel is the compaction's
  const CompactKernels &K = part ? kPartition : kCompact;
  if (n == 0) {
    int64_t zero = 0;
    void *zargs[] = {&count, &zero};
    hipError_t e = hipLaunchKernel(kCompact.set_count, dim3(1), dim3(1), zargs, 0, stream);
    return e == hipSuccess ? SCAN_SUCCESS : hip_fail(e);
  }
  const int64_t tile = (int64_t)K.block * K.items;
  const int64_t T = tiles_for(n, tile);
  Workspace *ws = nullptr;
  if (T > 1) {
    s = stream_ws(dev, stream, T, &ws);
    if (s != SCAN_SUCCESS) return s;
  }
  // the predicate as the kernel's one compare: "nonzero" is an unsigned x > 0
  int kind = kPkUnsigned;
  if (predicate == SCAN_PRED_GREATER) kind = dt == SCAN_I32 ? kPkSigned : (dt == SCAN_F32 ? kPkFloat : kPkUnsigned);
  const uint32_t thr = predicate == SCAN_PRED_GREATER ? threshold : 0u;
  const void *fn = K.tiles[kind][((uintptr_t)in & 15u) == 0 ? 1 : 0];
  const int64_t grid = std::min<int64_t>(T, resident_grid(fn, K.block, di.cus, 0, 100));
  CompactArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k.in = in;
  a.k.out = out;
  a.k.n = n;
  a.k.tiles = T;
  a.k.hdr = ws ? ws->hdr : nullptr;
  a.k.status = ws ? ws->status : nullptr;
  a.k.capacity = ws ? ws->capacity : 0;
  a.k.total_acquires = (uint64_t)(T + grid);   // every workgroup also takes one tile past the end
  {
    std::lock_guard<std::mutex> lk(g_mu);
    a.k.spin_limit = g_spin_limit;
  }
  a.k.err = ws ? ws->err : nullptr;
  a.count = count;
  a.thr = thr;
  void *args[] = {&a};
  hipError_t e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(K.block), args, 0, stream);
  return e == hipSuccess ? SCAN_SUCCESS : hip_fail(e);
}

// Per-segment launches (comparator).  host_offsets are host memory.
scan_status_t looped(const void *in, void *out, const int64_t *host_offsets, int32_t S,
                     scan_dtype_t dt, uint32_t flags, hipStream_t stream, Workspace *ws) {
  int r = check_dtype((int)dt);
  if (r == kOk) r = check_flags(flags);
  if (r == kOk) r = check_operator((int)dt, flags);
  if (r != kOk) return st(r);
  if (S < 0 || (S > 0 && !host_offsets)) return SCAN_ERROR_INVALID_VALUE;
  if (S == 0) return SCAN_SUCCESS;
  const int64_t n = host_offsets[S];
  if (host_offsets[0] != 0) return SCAN_ERROR_INVALID_VALUE;
  for (int32_t s = 0; s < S; ++s)
    if (host_offsets[s + 1] < host_offsets[s]) return SCAN_ERROR_INVALID_VALUE;
  r = check_flat(in, out, n);
  if (r != kOk) return st(r);
  ensure_init();
  const char *pi = static_cast<const char *>(in);
  char *po = static_cast<char *>(out);
  for (int32_t s = 0; s < S; ++s) {
    const int64_t lo = host_offsets[s], len = host_offsets[s + 1] - lo;
    if (len == 0) continue;
    Call c = make_call(pi + 4 * lo, po + 4 * lo, len, dt, false, flags, nullptr, 0);
    scan_status_t e = launch(c, stream, ws, -1);
    if (e != SCAN_SUCCESS) return e;
  }
  return SCAN_SUCCESS;
}

// ---------------------------------------------------------------- graphs
struct GraphObj {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Workspace ws;
  uint32_t *err_host = nullptr;   // the graph's own error word
  uint32_t *err_dev = nullptr;
};

void graph_free(GraphObj *g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  ws_free(&g->ws);
  err_free(&g->err_host, &g->err_dev);
  delete g;
}

template <class Enqueue>
scan_status_t capture(int64_t need_tiles, hipStream_t stream, Enqueue enqueue, void **out) {
  if (!out) return SCAN_ERROR_INVALID_VALUE;
  *out = nullptr;
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  GraphObj *g = new GraphObj();
  s = err_alloc(&g->err_host, &g->err_dev);
  if (s == SCAN_SUCCESS) s = ws_alloc(&g->ws, dev, std::max<int64_t>(need_tiles, 2), stream);
  if (s != SCAN_SUCCESS) {
    graph_free(g);
    return s;
  }
  g->ws.err = g->err_dev;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) {
    graph_free(g);
    return hip_fail(e);
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = enqueue(cs, &g->ws);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (s == SCAN_SUCCESS && e2 != hipSuccess) s = hip_fail(e2);
    g->graph = graph;
    if (s == SCAN_SUCCESS) {
      e2 = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
      if (e2 != hipSuccess) s = hip_fail(e2);
    }
  } else {
    s = hip_fail(e);
  }
  (void)hipStreamDestroy(cs);
  if (s != SCAN_SUCCESS) {
    graph_free(g);
    return s;
  }
  *out = g;
  return SCAN_SUCCESS;
}

// ---------------------------------------------------------------- tune file
std::string default_tune_path() {
  const char *env = std::getenv("MI355SCAN_TUNE_FILE");
  if (env && *env) return env;
  Dl_info info;
  if (dladdr((void *)&default_tune_path, &info) && info.dli_fname) {
    std::string so = info.dli_fname;
    const size_t slash = so.rfind('/');
    const std::string dir = slash == std::string::npos ? "." : so.substr(0, slash);
    return dir + "/tune/gfx950.json";
  }
  return "";
}

// Reads the integer after "key": inside [b, e); returns false if absent.
bool json_int(const std::string &s, size_t b, size_t e, const char *key, long *out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k, b);
  if (p == std::string::npos || p >= e) return false;
  p = s.find(':', p + k.size());
  if (p == std::string::npos || p >= e) return false;
  ++p;
  while (p < e && (s[p] == ' ' || s[p] == '\t')) ++p;
  char *end = nullptr;
  const long v = std::strtol(s.c_str() + p, &end, 10);
  if (end == s.c_str() + p) return false;
  *out = v;
  return true;
}

bool json_str(const std::string &s, size_t b, size_t e, const char *key, std::string *out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k, b);
  if (p == std::string::npos || p >= e) return false;
  p = s.find('"', s.find(':', p + k.size()));
  if (p == std::string::npos || p >= e) return false;
  const size_t q = s.find('"', p + 1);
  if (q == std::string::npos || q >= e) return false;
  *out = s.substr(p + 1, q - p - 1);
  return true;
}

// Each entry: {"op": "int"|"f32", "segmented": 0|1, "log2n": b, "config": c,
// "block": B, "items": I}; entries whose block/items disagree with config c of
// this build are ignored.
scan_status_t parse_tune(const std::string &text) {
  int table[2][2][kBuckets];
  for (auto &a : table)
    for (auto &b : a)
      for (int &c : b) c = -1;
  size_t pos = text.find("\"entries\"");
  if (pos == std::string::npos) return SCAN_ERROR_INVALID_VALUE;
  for (;;) {
    const size_t b = text.find('{', pos);
    if (b == std::string::npos) break;
    const size_t e = text.find('}', b);
    if (e == std::string::npos) break;
    pos = e + 1;
    std::string op;
    long seg = 0, bucket = 0, cfg = 0, block = 0, items = 0;
    if (!json_str(text, b, e, "op", &op) || !json_int(text, b, e, "segmented", &seg) ||
        !json_int(text, b, e, "log2n", &bucket) || !json_int(text, b, e, "config", &cfg) ||
        !json_int(text, b, e, "block", &block) || !json_int(text, b, e, "items", &items))
      continue;
    if (cfg < 0 || cfg >= kNumConfigs || bucket < 0 || bucket >= kBuckets) continue;
    const KernelShape &sh = kShapes[kConfigs[cfg].shape];
    if (sh.block != block || sh.items != items) continue;
    const int oc = op == "f32" ? 1 : (op == "int" ? 0 : -1);
    if (oc < 0) continue;
    table[oc][seg ? 1 : 0][bucket] = (int)cfg;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  std::memcpy(g_table, table, sizeof(table));
  return SCAN_SUCCESS;
}

scan_status_t load_tune(const char *path) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return SCAN_ERROR_INVALID_VALUE;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
  std::fclose(f);
  return parse_tune(text);
}

void load_default_tune_file() {
  const std::string p = default_tune_path();
  if (!p.empty()) (void)load_tune(p.c_str());
}

}  // namespace
}  // namespace mi355scan

using namespace mi355scan;

extern "C" {

scan_status_t scan_flat(const void *in, void *out, int64_t n, scan_dtype_t dtype, uint32_t flags,
                        hipStream_t stream) {
  return flat(in, out, n, dtype, flags, stream);
}

scan_status_t scan_stream_ceiling(const void *in, void *out, int64_t n, int32_t config, hipStream_t stream) {
  return stream_ceiling(in, out, n, config, stream);
}

scan_status_t scan_flat_noalloc(const void *in, void *out, int64_t n, scan_dtype_t dtype, uint32_t flags,
                                hipStream_t stream) {
  return flat_noalloc(in, out, n, dtype, flags, stream);
}

scan_status_t scan_inclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  return flat(in, out, n, SCAN_I32, 0u, s);
}
scan_status_t scan_inclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s) {
  return flat(in, out, n, SCAN_U32, 0u, s);
}
scan_status_t scan_inclusive_f32(const float *in, float *out, int64_t n, hipStream_t s) {
  return flat(in, out, n, SCAN_F32, 0u, s);
}
scan_status_t scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  return flat(in, out, n, SCAN_I32, SCAN_EXCLUSIVE, s);
}
scan_status_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s) {
  return flat(in, out, n, SCAN_U32, SCAN_EXCLUSIVE, s);
}
scan_status_t scan_exclusive_f32(const float *in, float *out, int64_t n, hipStream_t s) {
  return flat(in, out, n, SCAN_F32, SCAN_EXCLUSIVE, s);
}

scan_status_t scan_segmented_batch(const void *in, void *out, const int64_t *offsets,
                                   int32_t num_segments, int64_t n, scan_dtype_t dtype,
                                   uint32_t flags, hipStream_t stream) {
  return segmented(in, out, offsets, num_segments, n, dtype, flags, stream, nullptr, -1);
}

scan_status_t scan_f32_backward(const float *grad_out, float *grad_in, int64_t n,
                                const int64_t *offsets, int32_t num_segments, hipStream_t stream) {
  if (!offsets) return flat(grad_out, grad_in, n, SCAN_F32, SCAN_REVERSE, stream);
  return segmented(grad_out, grad_in, offsets, num_segments, n, SCAN_F32, SCAN_REVERSE, stream,
                   nullptr, -1);
}

scan_status_t scan_two_pass(const void *in, void *out, int64_t n, scan_dtype_t dtype, uint32_t flags,
                            int32_t method, int64_t partition, hipStream_t stream) {
  return two_pass(in, out, n, dtype, flags, method, partition, stream);
}

scan_status_t scan_compact(const void *in, void *out, int64_t n, scan_dtype_t dtype, int32_t predicate,
                           uint32_t threshold, int64_t *count, hipStream_t stream) {
  return compact(in, out, n, dtype, predicate, threshold, count, stream);
}

scan_status_t scan_partition(const void *in, void *out, int64_t n, scan_dtype_t dtype, int32_t predicate,
                             uint32_t threshold, int64_t *count, hipStream_t stream) {
  return compact(in, out, n, dtype, predicate, threshold, count, stream, true);
}

scan_status_t scan_reserve(int64_t max_n, hipStream_t stream) {
  if (max_n < 0) return SCAN_ERROR_INVALID_VALUE;
  if (max_n == 0) return SCAN_SUCCESS;
  ensure_init();
  int dev = 0;
  DeviceInfo di;
  scan_status_t s = current_device(&dev, &di);
  if (s != SCAN_SUCCESS) return s;
  Workspace *w = nullptr;
  return stream_ws(dev, stream, tiles_for(max_n, min_tile()), &w);
}

scan_status_t scan_release(hipStream_t stream) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, SCAN_ERROR_NOT_SUPPORTED);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(std::make_pair(dev, stream));
  if (it == g_ws.end()) return SCAN_SUCCESS;
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e);
  StreamState &ss = it->second;
  ws_free(&ss.ws);
  for (Workspace &w : ss.retired) ws_free(&w);
  err_free(&ss.err_host, &ss.err_dev);
  g_ws.erase(it);
  return SCAN_SUCCESS;
}

scan_status_t scan_segmented_graph_create(const void *in, void *out, const int64_t *offsets,
                                          int32_t num_segments, int64_t n, scan_dtype_t dtype,
                                          uint32_t flags, hipStream_t stream, void **graph) {
  int r = check_dtype((int)dtype);
  if (r == kOk) r = check_flags(flags);
  if (r == kOk) r = check_segmented(in, out, offsets, num_segments, n);
  if (r == kOk) r = check_operator((int)dtype, flags);
  if (r != kOk) return st(r);
  ensure_init();
  const int cfg = select_config(opclass_of(dtype), true, n);
  Call c = make_call(in, out, n, dtype, true, flags, offsets, num_segments);
  const int64_t need = call_tiles(c, cfg);
  return capture(need, stream,
                 [&](hipStream_t cs, Workspace *ws) {
                   return segmented(in, out, offsets, num_segments, n, dtype, flags, cs, ws, cfg);
                 },
                 graph);
}

scan_status_t scan_looped_graph_create(const void *in, void *out, const int64_t *host_offsets,
                                       int32_t num_segments, scan_dtype_t dtype, uint32_t flags,
                                       hipStream_t stream, void **graph) {
  if (num_segments < 0 || (num_segments > 0 && !host_offsets)) return SCAN_ERROR_INVALID_VALUE;
  ensure_init();
  // tiles of the largest launch, sized with the pointers each launch gets
  // (their alignment picks the kernel shape and so the tile size)
  const char *pi = static_cast<const char *>(in);
  char *po = static_cast<char *>(out);
  int64_t need = 2;
  for (int32_t s = 0; s < num_segments; ++s) {
    const int64_t lo = host_offsets[s], len = host_offsets[s + 1] - lo;
    if (len > 0) {
      Call c = make_call(pi + 4 * lo, po + 4 * lo, len, dtype, false, flags, nullptr, 0);
      need = std::max(need, call_tiles(c, select_config(c.opclass, false, len)));
    }
  }
  return capture(need, stream,
                 [&](hipStream_t cs, Workspace *ws) {
                   return looped(in, out, host_offsets, num_segments, dtype, flags, cs, ws);
                 },
                 graph);
}

scan_status_t scan_graph_launch(void *graph, hipStream_t stream) {
  if (!graph) return SCAN_ERROR_INVALID_VALUE;
  GraphObj *g = static_cast<GraphObj *>(graph);
  if (take_error(g->err_host)) return SCAN_ERROR_TIMEOUT;   // an earlier replay gave up a wait
  hipError_t e = hipGraphLaunch(g->exec, stream);
  return e == hipSuccess ? SCAN_SUCCESS : hip_fail(e);
}

scan_status_t scan_graph_check_device_error(void *graph) {
  if (!graph) return SCAN_ERROR_INVALID_VALUE;
  return take_error(static_cast<GraphObj *>(graph)->err_host) ? SCAN_ERROR_TIMEOUT : SCAN_SUCCESS;
}

scan_status_t scan_graph_destroy(void *graph) {
  if (!graph) return SCAN_ERROR_INVALID_VALUE;
  GraphObj *g = static_cast<GraphObj *>(graph);
  (void)hipDeviceSynchronize();
  graph_free(g);
  return SCAN_SUCCESS;
}

scan_status_t scan_segmented_looped(const void *in, void *out, const int64_t *host_offsets,
                                    int32_t num_segments, scan_dtype_t dtype, uint32_t flags,
                                    hipStream_t stream) {
  return looped(in, out, host_offsets, num_segments, dtype, flags, stream, nullptr);
}

int32_t scan_num_configs(void) { return kNumConfigs; }

scan_status_t scan_config_info(int32_t config, int32_t *block, int32_t *items, int32_t *nontemporal,
                               int32_t *mode, int32_t *per_cu, int32_t *cu_pct) {
  if (config < 0 || config >= kNumConfigs) return SCAN_ERROR_INVALID_VALUE;
  const KernelShape &sh = kShapes[kConfigs[config].shape];
  if (block) *block = sh.block;
  if (items) *items = sh.items;
  if (nontemporal) *nontemporal = sh.nontemporal;
  if (mode) *mode = kConfigs[config].mode;
  if (per_cu) *per_cu = kConfigs[config].per_cu;
  if (cu_pct) *cu_pct = kConfigs[config].cu_pct;
  return SCAN_SUCCESS;
}

scan_status_t scan_force_config(int32_t config) {
  if (config < -1 || config >= kNumConfigs) return SCAN_ERROR_INVALID_VALUE;
  std::lock_guard<std::mutex> lk(g_mu);
  g_forced = config;
  return SCAN_SUCCESS;
}

int32_t scan_selected_config(scan_dtype_t dtype, uint32_t flags, int32_t segmented, int64_t n) {
  (void)flags;
  if (check_dtype((int)dtype) != kOk || n < 0) return -1;
  ensure_init();
  return select_config(opclass_of(dtype), segmented != 0, n);
}

scan_status_t scan_autotune(const void *in, void *out, int64_t n, const int64_t *offsets,
                            int32_t num_segments, scan_dtype_t dtype, uint32_t flags, int32_t reps,
                            hipStream_t stream, int32_t *best) {
  int r = check_dtype((int)dtype);
  if (r == kOk) r = check_flags(flags);
  const bool seg = offsets != nullptr;
  if (r == kOk) r = seg ? check_segmented(in, out, offsets, num_segments, n) : check_flat(in, out, n);
  if (r == kOk) r = check_operator((int)dtype, flags);
  if (r != kOk) return st(r);
  if (n == 0 || reps < 1) return SCAN_ERROR_INVALID_VALUE;
  ensure_init();
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return hip_fail(e);
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e);
  }
  Call c = make_call(in, out, n, dtype, seg, flags, offsets, num_segments);
  float best_ms = 1e30f, best_dyn_ms = 1e30f;
  int best_cfg = -1, best_dyn = -1;
  scan_status_t s = SCAN_SUCCESS;
  for (int cfg = 0; cfg < kNumConfigs && s == SCAN_SUCCESS; ++cfg) {
    std::vector<float> times;
    for (int i = 0; i < reps + 1 && s == SCAN_SUCCESS; ++i) {
      if ((e = hipEventRecord(e0, stream)) != hipSuccess) { s = hip_fail(e); break; }
      s = launch(c, stream, nullptr, cfg);
      if (s != SCAN_SUCCESS) break;
      if ((e = hipEventRecord(e1, stream)) != hipSuccess) { s = hip_fail(e); break; }
      if ((e = hipEventSynchronize(e1)) != hipSuccess) { s = hip_fail(e); break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (i > 0) times.push_back(ms);   // first run warms up
    }
    if (s != SCAN_SUCCESS) break;
    std::sort(times.begin(), times.end());
    const float med = times[times.size() / 2];
    if (med < best_ms) {
      best_ms = med;
      best_cfg = cfg;
    }
    const int mode = kConfigs[cfg].mode;
    if ((mode == kModeCounter || mode == kModePersistent) && med < best_dyn_ms) {
      best_dyn_ms = med;
      best_dyn = cfg;
    }
  }
  if (best_dyn >= 0 && best_cfg != best_dyn && !(best_ms < best_dyn_ms * (1.0f - kOrderedMargin)))
    best_cfg = best_dyn;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != SCAN_SUCCESS) return s;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[c.opclass][seg ? 1 : 0][bucket_of(n)] = best_cfg;
  }
  if (best) *best = best_cfg;
  return SCAN_SUCCESS;
}

scan_status_t scan_tune_save(const char *path) {
  if (!path) return SCAN_ERROR_INVALID_VALUE;
  ensure_init();
  FILE *f = std::fopen(path, "wb");
  if (!f) return SCAN_ERROR_INVALID_VALUE;
  std::fprintf(f, "{\n  \"arch\": \"gfx950\",\n  \"format\": 1,\n  \"entries\": [");
  bool first = true;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int oc = 0; oc < 2; ++oc)
    for (int sg = 0; sg < 2; ++sg)
      for (int b = 0; b < kBuckets; ++b) {
        const int cfg = g_table[oc][sg][b];
        if (cfg < 0) continue;
        const KernelShape &sh = kShapes[kConfigs[cfg].shape];
        std::fprintf(f,
                     "%s\n    {\"op\": \"%s\", \"segmented\": %d, \"log2n\": %d, \"config\": %d, "
                     "\"block\": %d, \"items\": %d, \"nontemporal\": %d, \"mode\": %d}",
                     first ? "" : ",", oc ? "f32" : "int", sg, b, cfg, sh.block, sh.items,
                     sh.nontemporal, kConfigs[cfg].mode);
        first = false;
      }
  std::fprintf(f, "\n  ]\n}\n");
  std::fclose(f);
  return SCAN_SUCCESS;
}

scan_status_t scan_tune_load(const char *path) {
  if (!path) return SCAN_ERROR_INVALID_VALUE;
  ensure_init();
  return load_tune(path);
}

const char *scan_status_string(scan_status_t status) {
  switch (status) {
    case SCAN_SUCCESS: return "success";
    case SCAN_ERROR_INVALID_VALUE: return "invalid value";
    case SCAN_ERROR_OVERLAP: return "input and output overlap without being equal";
    case SCAN_ERROR_OUT_OF_MEMORY: return "out of device memory";
    case SCAN_ERROR_LAUNCH: return "HIP call failed";
    case SCAN_ERROR_NOT_SUPPORTED: return "no supported (gfx950) device";
    case SCAN_ERROR_CAPTURE: return "workspace growth refused during stream capture";
    case SCAN_ERROR_TIMEOUT: return "device wait exceeded its spin limit";
  }
  return "unknown status";
}

int32_t scan_last_hip_error(void) { return t_last_hip; }

scan_status_t scan_set_spin_limit(uint32_t limit) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_spin_limit = limit ? limit : kDefaultSpinLimit;
  return SCAN_SUCCESS;
}

scan_status_t scan_check_device_error(hipStream_t stream) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, SCAN_ERROR_NOT_SUPPORTED);
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e);
  scan_status_t s = stream_pending(dev, stream);
  // the device's allocation-free workspace (scan_flat_noalloc), if set up:
  // its error word is device memory, read and cleared by plain copies
  if (Workspace *sw = scratch_ws_if_set(dev)) {
    uint32_t v = 0u;
    e = hipMemcpy(&v, &sw->hdr->error, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    if (v) {
      const uint32_t zero = 0u;
      e = hipMemcpy(&sw->hdr->error, &zero, sizeof(zero), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e);
      s = SCAN_ERROR_TIMEOUT;
    }
  }
  return s;
}

}  // extern "C"
