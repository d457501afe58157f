// jsidx_noalloc.hip -- jsidx_build without any device allocation (see
// include/jsidx.h): the same launch as jsidx_build over a workspace held in a
// file-scope device array.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "jsidx.h"
#include "jsidx_doc.h"
#include "jsidx_host.h"

namespace jsidx {

// ---- a workspace that needs no allocation ----------------------------------
// jsidx_build_noalloc runs the one-document kernel over a workspace in a
// file-scope device array: the header (counters, epoch, diagnostic) and the
// kernel's region (tile descriptors, block words and counters) right after it;
// that kernel keeps its masks in LDS, so nothing else is needed.  Each device
// holds its own copy until the process ends; its device address is taken once
// per device (hipGetSymbolAddress) and only that address is ever passed to a
// kernel.
constexpr uint64_t kStaticTiles = (JSIDX_NOALLOC_MAX_LEN + 15 + kTileBytes - 1) / kTileBytes;
constexpr uint64_t kStaticDocOff = 256;
constexpr uint64_t kStaticWsBytes = (kStaticDocOff + doc_region_bytes(kStaticTiles) + 255) & ~(uint64_t)255;
static_assert(sizeof(Workspace) <= kStaticDocOff, "the header fits before the region");
static_assert(kStaticWsBytes <= (1ull << 20), "the static workspace stays modest");
static __device__ __align__(256) uint8_t scratch[kStaticWsBytes];

struct StaticWs {
  bool ready;
  void* ptr;  // device address of `scratch` on this device
};
StaticWs g_static[64];

// Zeroes n 64-bit words (a kernel, so that a graph capture records no memset).
__global__ void __launch_bounds__(256) zero_words(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = 0ull;
}

// The static workspace of the current device, set up on first use: its
// address, and all of it zeroed on `stream`.  Caller holds g_mu.
int static_ws(hipStream_t stream, StreamWs* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  if (dev < 0 || dev >= 64) return JSIDX_E_HIP;
  StaticWs& s = g_static[dev];
  if (!s.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return JSIDX_E_HIP;
    (void)hipGetLastError();
    hipLaunchKernelGGL(zero_words, dim3(64), dim3(256), 0, stream, (uint64_t*)p, kStaticWsBytes / 8);
    if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
    s.ptr = p;
    s.ready = true;
  }
  *out = StreamWs{dev, stream, (Workspace*)s.ptr, kStaticTiles, true, kStaticDocOff};
  return JSIDX_OK;
}

}  // namespace jsidx

using namespace jsidx;

extern "C" {

int jsidx_build_noalloc(const uint8_t* buf, uint64_t len, uint32_t* out_idx, uint32_t* out_n, uint32_t* out_err,
                        jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!out_idx || !out_n || !out_err || (!buf && len)) return JSIDX_E_INVAL;
  if (len >= (1ull << 32)) return JSIDX_E_INVAL;
  if (len > JSIDX_NOALLOC_MAX_LEN) return JSIDX_E_TOO_LARGE;
  std::lock_guard<std::mutex> lk(g_mu);
  StreamWs e;
  const int rc = static_ws(stream, &e);
  if (rc) return rc;
  return launch_doc(buf, len, out_idx, out_n, out_err, stream, e);
}

}  // extern "C"
