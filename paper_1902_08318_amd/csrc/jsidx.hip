// jsidx.hip -- MI355X (gfx950) stage-1 JSON structural index (Langdale &
// Lemire, "Parsing Gigabytes of JSON per Second", Sec. 3.1) behind the C ABI
// of include/jsidx.h.
//
// One persistent launch indexes one document or a batch.  Work is cut into
// tiles of 2 to 16 rows of 2 KiB of the concatenated input (the tile size is
// chosen per launch from the input size); each wave of a workgroup of 8
// independent waves takes tiles in increasing order from a ticket counter.
// Inside a tile every lane owns one 32-byte segment per row and builds
// 32-bit class masks for it from bit planes (Sec. 3.1.2); escapes (Fig. 3),
// string ranges (Fig. 4) and pseudo-structural bytes (Fig. 5) are computed
// per segment, with the carries between segments resolved by wave ballots
// and the carries between tiles by a decoupled look-back over per-tile and
// per-block descriptors (the paper's per-block carries, elided in its
// footnote, become a scan).  Document starts reset all carries, so a batch
// of documents is one segmented scan.  Set bits are flattened into uint32
// positions per document (Sec. 3.1.4): a popcount per segment and a wave
// prefix sum give each bit its slot; the look-back gives each tile its base.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "jsidx.h"
#include "jsidx_doc.h"
#include "jsidx_host.h"
#include "jsidx_kernel.h"

namespace jsidx {

// Waves per SIMD the register budget is sized for (4: up to 128 VGPRs).
#ifndef JSIDX_WAVES_PER_EU
#define JSIDX_WAVES_PER_EU 4
#endif
template <int VAR>
__global__ void __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(JSIDX_WAVES_PER_EU)))
index_kernel(Args a) {
  index_tiles<false, VAR>(a);
}

// The same pass with the kept bytes (not white space outside strings) as output.
__global__ void __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(JSIDX_WAVES_PER_EU)))
minify_kernel(Args a) {
  index_tiles<true>(a);
}

// One document (jsidx_build): the kernel of jsidx_doc.h.
// Waves per SIMD of the one-document kernel (its LDS allows one workgroup of
// kDocWaves waves per compute unit).
#ifndef JSIDX_DOC_WAVES_PER_EU
#define JSIDX_DOC_WAVES_PER_EU (JSIDX_DOC_WAVES / 4)
#endif
template <int VAR>
__global__ void __launch_bounds__(kDocThreads) __attribute__((amdgpu_waves_per_eu(JSIDX_DOC_WAVES_PER_EU)))
doc_kernel(DocArgs a) {
  doc_tiles<VAR>(a);
}

// Checks a batch's offsets before its indexing launch (see offsets_check).
constexpr int kCheckThreads = 256;
__global__ void __launch_bounds__(kCheckThreads) offsets_check_kernel(const uint64_t* offsets, uint32_t ndocs,
                                                                     Workspace* ws) {
  offsets_check(offsets, ndocs, ws, kCheckThreads);
}

// ---------------------------------------------------------------------------
// host side
std::mutex g_mu;
std::vector<StreamWs> g_ws;
uint64_t g_rows_tab[4];  // tile rows by size class (jsidx_set_tile_rows), 0 = default
uint32_t g_variant = 0;  // indexing kernel variant (jsidx_set_variant)
// Kernels by slot: the batch index kernel's variants 0, naive
// classification, loop prefix XOR, direct flatten; the minify kernel; then the
// one-document kernel's variants in the same order.
constexpr int kKernels = 9;
constexpr int kMinifySlot = 4;
constexpr int kDocSlot = 5;
const void* kernel_at(int k) {
  switch (k) {
    case 0: return reinterpret_cast<const void*>(&index_kernel<0>);
    case 1: return reinterpret_cast<const void*>(&index_kernel<kVarNaiveClassify>);
    case 2: return reinterpret_cast<const void*>(&index_kernel<kVarXorLoop>);
    case 3: return reinterpret_cast<const void*>(&index_kernel<kVarDirectFlatten>);
    case 4: return reinterpret_cast<const void*>(&minify_kernel);
    case 5: return reinterpret_cast<const void*>(&doc_kernel<0>);
    case 6: return reinterpret_cast<const void*>(&doc_kernel<kVarNaiveClassify>);
    case 7: return reinterpret_cast<const void*>(&doc_kernel<kVarXorLoop>);
    default: return reinterpret_cast<const void*>(&doc_kernel<kVarDirectFlatten>);
  }
}
int kernel_threads(int k) { return k >= kDocSlot ? kDocThreads : kGroupThreads; }
int slot_of_variant(uint32_t v) {
  return v == 0 ? 0 : v == (uint32_t)kVarNaiveClassify ? 1 : v == (uint32_t)kVarXorLoop ? 2
       : v == (uint32_t)kVarDirectFlatten ? 3 : -1;
}
int g_slots[kKernels][64];  // resident workgroups per kernel and device (0 = not queried)

uint64_t tiles_for(uint64_t total_len) {
  uint64_t t = (total_len + 15 + kTileBytes - 1) / kTileBytes;
  return t ? t : 1;
}

size_t ws_bytes_for_tiles(uint64_t tiles) { return (size_t)stream_ws_bytes(tiles); }

int slots_for_device(int dev, int kernel) {
  if (dev < 0 || dev >= 64) return 1024;
  int& slots = g_slots[kernel][dev];
  if (slots) return slots;
  int per_cu = 0;
  const hipError_t rc =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_at(kernel), kernel_threads(kernel), 0);
  if (rc != hipSuccess || per_cu < 1) per_cu = 1;
  hipDeviceProp_t prop;
  int cus = 256;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  slots = per_cu * cus;
  return slots;
}

// A zeroed device allocation for a workspace of `tiles` largest tiles, or
// nullptr (nothing left allocated) if any step fails.
Workspace* alloc_ws(hipStream_t stream, uint64_t tiles) {
  void* p = nullptr;
  const size_t bytes = ws_bytes_for_tiles(tiles);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();  // not left behind for the next launch check
    return nullptr;
  }
  if (hipMemsetAsync(p, 0, bytes, stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
    (void)hipFree(p);
    (void)hipGetLastError();
    return nullptr;
  }
  return (Workspace*)p;
}

// Find or grow the workspace of (current device, stream).  Caller holds g_mu.
// A failed growth leaves the stream without a workspace (its entry is
// removed), so no later launch can see a stale capacity with no memory.
int get_ws(hipStream_t stream, uint64_t need_tiles, bool grow, StreamWs** out) {
  int dev = 0;
  *out = nullptr;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  bool reserved = false;
  for (size_t i = 0; i < g_ws.size(); i++) {
    StreamWs& e = g_ws[i];
    if (e.device == dev && e.stream == stream) {
      if (e.cap_tiles >= need_tiles || !grow) { *out = &e; return JSIDX_OK; }
      if (hipStreamSynchronize(stream) != hipSuccess) return JSIDX_E_HIP;
      reserved = e.reserved;
      (void)hipFree(e.ws);
      g_ws.erase(g_ws.begin() + (long)i);
      break;
    }
  }
  if (!grow) return JSIDX_OK;
  Workspace* p = alloc_ws(stream, need_tiles);
  if (!p) return JSIDX_E_NOWORKSPACE;
  g_ws.push_back(StreamWs{dev, stream, p, need_tiles, reserved, doc_region_offset(need_tiles)});
  *out = &g_ws.back();
  return JSIDX_OK;
}

// Launch over a workspace of e->cap_tiles largest tiles.  span >= 0: the
// bytes from the 16-byte granule holding the first byte to the end (one
// document, known here), so the tile size and the grid fit the input;
// span < 0 (batch, sizes on the device): the grid covers the workspace and
// the kernel picks the tile size.
int launch(Args& a, hipStream_t stream, const StreamWs& e, int64_t span, bool minify) {
  int dev = 0;
  if (!e.ws) return JSIDX_E_NOWORKSPACE;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  const int kernel = minify ? kMinifySlot : slot_of_variant(g_variant);
  const uint64_t slots = (uint64_t)slots_for_device(dev, kernel);
  a.ws = e.ws;
  a.cap_tiles = desc_slots(e.cap_tiles);
  a.cap_rows = e.cap_tiles * (uint64_t)kRows;
  uint64_t tiles = a.cap_tiles;
  a.rows = 0;
  for (int i = 0; i < 4; i++) a.rows_tab[i] = g_rows_tab[i];
  if (span >= 0) {
    a.rows = rows_for(span, slots * kWaves, a.rows_tab);
    const uint64_t tb = (uint64_t)a.rows * kRowBytes;
    tiles = span > 0 ? ((uint64_t)span + tb - 1) / tb : 1;
  }
  const uint64_t groups = (tiles + kWaves - 1) / kWaves;
  uint64_t grid = groups < slots ? groups : slots;
  if (grid < 1) grid = 1;
  a.fill_waves = (uint32_t)(grid * kWaves);
  (void)hipGetLastError();  // the check after the launch sees only the launch
  switch (kernel) {
    case 0: hipLaunchKernelGGL(index_kernel<0>, dim3((uint32_t)grid), dim3(kGroupThreads), 0, stream, a); break;
    case 1:
      hipLaunchKernelGGL(index_kernel<kVarNaiveClassify>, dim3((uint32_t)grid), dim3(kGroupThreads), 0, stream, a);
      break;
    case 2: hipLaunchKernelGGL(index_kernel<kVarXorLoop>, dim3((uint32_t)grid), dim3(kGroupThreads), 0, stream, a); break;
    case 3:
      hipLaunchKernelGGL(index_kernel<kVarDirectFlatten>, dim3((uint32_t)grid), dim3(kGroupThreads), 0, stream, a);
      break;
    default: hipLaunchKernelGGL(minify_kernel, dim3((uint32_t)grid), dim3(kGroupThreads), 0, stream, a); break;
  }
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}

// One document with the kernel of jsidx_doc.h over workspace e.
int launch_doc(const uint8_t* buf, uint64_t len, uint32_t* out, uint32_t* out_n, uint32_t* out_err,
               hipStream_t stream, const StreamWs& e) {
  int dev = 0;
  if (!e.ws) return JSIDX_E_NOWORKSPACE;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  const int kernel = kDocSlot + slot_of_variant(g_variant);
  const uint64_t slots = (uint64_t)slots_for_device(dev, kernel);
  DocArgs a;
  a.base = buf ? buf : reinterpret_cast<const uint8_t*>(out);  // never read when len == 0
  a.len = len;
  a.out_idx = out;
  a.out_n = out_n;
  a.out_err = out_err;
  a.ws = e.ws;
  uint8_t* region = reinterpret_cast<uint8_t*>(e.ws) + e.doc_off;
  a.cap = doc_cap_for(e.cap_tiles);
  a.desc = reinterpret_cast<uint64_t*>(region);
  a.blk = a.desc + a.cap;
  a.bcnt = reinterpret_cast<uint32_t*>(a.blk + 2 * doc_blocks_for(a.cap));
  a.p0 = -(int64_t)((uintptr_t)a.base & 15u);
  a.ntiles = len ? ((int64_t)len - a.p0 + kDocTile - 1) / kDocTile : 0;
  const uint64_t groups = ((uint64_t)a.ntiles + kDocWaves - 1) / kDocWaves;
  uint64_t grid = groups < slots ? groups : slots;
  if (grid < 1) grid = 1;
  (void)hipGetLastError();
  switch (kernel) {
    case kDocSlot: hipLaunchKernelGGL(doc_kernel<0>, dim3((uint32_t)grid), dim3(kDocThreads), 0, stream, a); break;
    case kDocSlot + 1:
      hipLaunchKernelGGL(doc_kernel<kVarNaiveClassify>, dim3((uint32_t)grid), dim3(kDocThreads), 0, stream, a);
      break;
    case kDocSlot + 2:
      hipLaunchKernelGGL(doc_kernel<kVarXorLoop>, dim3((uint32_t)grid), dim3(kDocThreads), 0, stream, a);
      break;
    default:
      hipLaunchKernelGGL(doc_kernel<kVarDirectFlatten>, dim3((uint32_t)grid), dim3(kDocThreads), 0, stream, a);
      break;
  }
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}

}  // namespace jsidx

using namespace jsidx;

namespace jsidx {

int build_one(const uint8_t* buf, uint64_t len, uint32_t* out, uint32_t* out_n, uint32_t* out_err,
              hipStream_t stream, bool minify) {
  if (!out || !out_n || !out_err || (!buf && len)) return JSIDX_E_INVAL;
  if (len >= (1ull << 32)) return JSIDX_E_INVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  StreamWs* e = nullptr;
  uint64_t need = tiles_for(len);
  int rc = get_ws(stream, need, true, &e);
  if (rc) return rc;
  if (!minify) return launch_doc(buf, len, out, out_n, out_err, stream, *e);
  Args a;
  a.base = buf ? buf : reinterpret_cast<const uint8_t*>(out);  // never read when len == 0
  a.offsets = nullptr;
  a.len = len;
  a.ndocs = 1;
  a.out_idx = out;
  a.out_n = out_n;
  a.out_err = out_err;
  return launch(a, stream, *e, (int64_t)(len + ((uintptr_t)a.base & 15u)), minify);
}

int build_many(const uint8_t* bufs, const uint64_t* offsets, uint32_t ndocs, uint32_t* out, uint32_t* out_n,
               uint32_t* out_err, hipStream_t stream, bool minify) {
  if (!bufs || !offsets || !out || !out_n || !out_err || ndocs == 0) return JSIDX_E_INVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  StreamWs* e = nullptr;
  int rc = get_ws(stream, 0, false, &e);
  if (rc) return rc;
  if (!e || !e->reserved) {
    uint64_t ends[2];
    if (hipMemcpyAsync(&ends[0], offsets, 8, hipMemcpyDeviceToHost, stream) != hipSuccess) return JSIDX_E_HIP;
    if (hipMemcpyAsync(&ends[1], offsets + ndocs, 8, hipMemcpyDeviceToHost, stream) != hipSuccess) return JSIDX_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return JSIDX_E_HIP;
    uint64_t total = ends[1] > ends[0] ? ends[1] - ends[0] : 0;
    rc = get_ws(stream, tiles_for(total), true, &e);
    if (rc) return rc;
  }
  if (!e || !e->ws) return JSIDX_E_NOWORKSPACE;
  // the offsets are checked first; the indexing launch reads the verdict
  {
    uint64_t g = ((uint64_t)ndocs + kCheckThreads - 1) / kCheckThreads;
    if (g > 1024) g = 1024;
    (void)hipGetLastError();
    hipLaunchKernelGGL(offsets_check_kernel, dim3((uint32_t)g), dim3(kCheckThreads), 0, stream, offsets, ndocs, e->ws);
    if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  }
  Args a;
  a.base = bufs;
  a.offsets = offsets;
  a.len = 0;
  a.ndocs = ndocs;
  a.out_idx = out;
  a.out_n = out_n;
  a.out_err = out_err;
  return launch(a, stream, *e, -1, minify);
}

}  // namespace jsidx

#ifdef JSIDX_PROBE
namespace jsidx {
namespace prim {
__device__ uint64_t* g_probe;
}  // namespace prim
}  // namespace jsidx
#endif

extern "C" {

#ifdef JSIDX_PROBE
// Probe builds only: the buffer the tile events are written to (0: none).
int jsidx_probe_set(void* p) {
  uint64_t* v = (uint64_t*)p;
  return hipMemcpyToSymbol(HIP_SYMBOL(jsidx::prim::g_probe), &v, sizeof(v)) == hipSuccess ? 0 : -3;
}
#endif

int jsidx_build(const uint8_t* buf, uint64_t len, uint32_t* out_idx, uint32_t* out_n, uint32_t* out_err,
                jsidx_stream_t stream) {
  return build_one(buf, len, out_idx, out_n, out_err, (hipStream_t)stream, false);
}

int jsidx_build_batch(const uint8_t* bufs, const uint64_t* offsets, uint32_t ndocs, uint32_t* out_idx,
                      uint32_t* out_n, uint32_t* out_err, jsidx_stream_t stream) {
  return build_many(bufs, offsets, ndocs, out_idx, out_n, out_err, (hipStream_t)stream, false);
}

int jsidx_minify(const uint8_t* buf, uint64_t len, uint8_t* out, uint32_t* out_n, uint32_t* out_err,
                 jsidx_stream_t stream) {
  return build_one(buf, len, reinterpret_cast<uint32_t*>(out), out_n, out_err, (hipStream_t)stream, true);
}

int jsidx_minify_batch(const uint8_t* bufs, const uint64_t* offsets, uint32_t ndocs, uint8_t* out, uint32_t* out_n,
                       uint32_t* out_err, jsidx_stream_t stream) {
  return build_many(bufs, offsets, ndocs, reinterpret_cast<uint32_t*>(out), out_n, out_err, (hipStream_t)stream,
                    true);
}

int jsidx_reserve(uint64_t max_total_len, uint32_t max_ndocs, jsidx_stream_t stream_) {
  (void)max_ndocs;  // the workspace is sized by bytes only
  std::lock_guard<std::mutex> lk(g_mu);
  StreamWs* e = nullptr;
  int rc = get_ws((hipStream_t)stream_, tiles_for(max_total_len), true, &e);
  if (rc == JSIDX_OK) e->reserved = true;
  return rc;
}

size_t jsidx_workspace_bytes(uint64_t total_len, uint32_t ndocs) {
  (void)ndocs;
  return ws_bytes_for_tiles(tiles_for(total_len));
}

int jsidx_release(jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  for (size_t i = 0; i < g_ws.size(); i++) {
    if (g_ws[i].device == dev && g_ws[i].stream == stream) {
      if (hipStreamSynchronize(stream) != hipSuccess) return JSIDX_E_HIP;
      (void)hipFree(g_ws[i].ws);
      g_ws.erase(g_ws.begin() + (long)i);
      return JSIDX_OK;
    }
  }
  return JSIDX_OK;
}

int jsidx_stream_diag(jsidx_stream_t stream_, uint32_t* out_flags) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!out_flags) return JSIDX_E_INVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  StreamWs* e = nullptr;
  int rc = get_ws(stream, 0, false, &e);
  if (rc) return rc;
  *out_flags = 0;
  if (!e) return JSIDX_OK;
  if (hipStreamSynchronize(stream) != hipSuccess) return JSIDX_E_HIP;
  uint32_t v = 0;
  if (hipMemcpy(&v, &e->ws->diag, 4, hipMemcpyDeviceToHost) != hipSuccess) return JSIDX_E_HIP;
  if (v && hipMemset(&e->ws->diag, 0, 4) != hipSuccess) return JSIDX_E_HIP;
  *out_flags = v;
  return JSIDX_OK;
}

int jsidx_set_tile_rows(const uint8_t* rows_by_log2, uint32_t n) {
  if (n > 64 || (n && !rows_by_log2)) return JSIDX_E_INVAL;
  uint64_t tab[4] = {0, 0, 0, 0};
  for (uint32_t b = 0; b < n; b++) {
    const uint32_t r = rows_by_log2[b];
    uint32_t code = 0;
    if (r) {
      if (r < (uint32_t)kMinRows || r > (uint32_t)kRows || (r & (r - 1u))) return JSIDX_E_INVAL;
      code = (uint32_t)__builtin_ctz(r);
    }
    tab[b >> 4] |= (uint64_t)code << (4u * (b & 15u));
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < 4; i++) g_rows_tab[i] = tab[i];
  return JSIDX_OK;
}

int jsidx_set_variant(uint32_t variant) {
  if (slot_of_variant(variant) < 0) return JSIDX_E_INVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  g_variant = variant;
  return JSIDX_OK;
}

int jsidx_tile_rows(uint64_t span, uint32_t* out_rows) {
  if (!out_rows) return JSIDX_E_INVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  const uint64_t slots = (uint64_t)slots_for_device(dev, slot_of_variant(g_variant));
  *out_rows = rows_for((int64_t)span, slots * kWaves, g_rows_tab);
  return JSIDX_OK;
}

const char* jsidx_status_string(int status) {
  switch (status) {
    case JSIDX_OK: return "ok";
    case JSIDX_E_INVAL: return "invalid argument";
    case JSIDX_E_NOWORKSPACE: return "workspace allocation failed";
    case JSIDX_E_HIP: return "HIP runtime error";
    case JSIDX_E_TOO_LARGE: return "input too large for the workspace";
    default: return "unknown status";
  }
}

}  // extern "C"
