// jsidx_scopes.hip -- the scope links of a document's structural index (the
// tape's scope links, Sec. 3, Fig. 2) behind jsidx_scopes of include/jsidx.h.
// The kernel bodies and the method are in jsidx_scopes.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "jsidx.h"
#include "jsidx_scopes.h"

namespace jsidx {

__global__ void __launch_bounds__(kScopeThreads) scope_chunk_fn_kernel(ScopeArgs a) { scope_chunk_fn(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_scan_kernel(ScopeArgs a) { scope_scan(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_levels_kernel(ScopeArgs a) { scope_levels(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_local_kernel(ScopeArgs a) { scope_local(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_far_kernel(ScopeArgs a) { scope_far(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_check_kernel(ScopeArgs a) { scope_check(a); }

namespace {

constexpr uint32_t kFarGroups = 512;  // workgroups of the last kernel (4 waves each)

struct ScopeWs {
  int device;
  hipStream_t stream;
  void* mem;
  uint64_t bytes;
};
std::mutex g_smu;
std::vector<ScopeWs> g_sws;

// The scope workspace of (current device, stream), grown to `bytes`.
int scope_ws(hipStream_t stream, uint64_t bytes, void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  for (auto& e : g_sws) {
    if (e.device != dev || e.stream != stream) continue;
    if (e.bytes < bytes) {
      if (hipStreamSynchronize(stream) != hipSuccess) return JSIDX_E_HIP;
      (void)hipFree(e.mem);
      e.mem = nullptr;
      e.bytes = 0;
      if (hipMalloc(&e.mem, bytes) != hipSuccess) return JSIDX_E_NOWORKSPACE;
      e.bytes = bytes;
    }
    *out = e.mem;
    return JSIDX_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return JSIDX_E_NOWORKSPACE;
  g_sws.push_back(ScopeWs{dev, stream, p, bytes});
  *out = p;
  return JSIDX_OK;
}

}  // namespace
}  // namespace jsidx

using namespace jsidx;

extern "C" int jsidx_scopes(const uint8_t* buf, uint64_t len, const uint32_t* idx, uint32_t n, uint32_t* out_match,
                            uint32_t* out_err, jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!out_err || (n && (!buf || !idx || !out_match))) return JSIDX_E_INVAL;
  if (len >= (1ull << 32)) return JSIDX_E_INVAL;
  const ScopeLayout L = scope_layout(n);
  std::lock_guard<std::mutex> lk(g_smu);
  void* mem = nullptr;
  int rc = scope_ws(stream, L.total, &mem);
  if (rc) return rc;
  uint8_t* m = static_cast<uint8_t*>(mem);
  ScopeArgs a;
  a.buf = buf ? buf : reinterpret_cast<const uint8_t*>(out_err);  // never read when n == 0
  a.len = len;
  a.idx = idx;
  a.n = n;
  a.nchunks = (uint32_t)((n + (uint64_t)kScopeChunk - 1) / kScopeChunk);
  a.match = out_match;
  a.err = out_err;
  a.chunk_fn = reinterpret_cast<uint2*>(m + L.chunk_fn);
  a.in_depth = reinterpret_cast<uint2*>(m + L.in_depth);
  a.chunk_min = reinterpret_cast<uint32_t*>(m + L.chunk_min);
  a.qcount = reinterpret_cast<uint32_t*>(m + L.qcount);
  a.lev = reinterpret_cast<uint32_t*>(m + L.lev);
  a.queue = reinterpret_cast<uint32_t*>(m + L.queue);
  a.kind = m + L.kind;
  const dim3 block(kScopeThreads);
  if (a.nchunks) hipLaunchKernelGGL(scope_chunk_fn_kernel, dim3(a.nchunks), block, 0, stream, a);
  hipLaunchKernelGGL(scope_scan_kernel, dim3(1), block, 0, stream, a);
  if (a.nchunks) {
    hipLaunchKernelGGL(scope_levels_kernel, dim3(a.nchunks), block, 0, stream, a);
    hipLaunchKernelGGL(scope_local_kernel, dim3(a.nchunks), block, 0, stream, a);
    hipLaunchKernelGGL(scope_far_kernel, dim3(kFarGroups), block, 0, stream, a);
    hipLaunchKernelGGL(scope_check_kernel, dim3(a.nchunks), block, 0, stream, a);
  }
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}
