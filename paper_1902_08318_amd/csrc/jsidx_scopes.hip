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

// the fold waits on its gathers: eight waves per SIMD keep more of them in
// flight (57 registers, no spills)
template <bool B>
__global__ void __launch_bounds__(kScopeThreads) __attribute__((amdgpu_waves_per_eu(8))) scope_chunk_fn_kernel(ScopeArgs a) {
  scope_chunk_fn<B>(a);
}
template <bool B>
__global__ void __launch_bounds__(kScopeThreads) scope_scan_kernel(ScopeArgs a) { scope_scan<B>(a); }
template <bool B>
__global__ void __launch_bounds__(kScopeThreads) scope_levels_kernel(ScopeArgs a) { scope_levels<B>(a); }
template <bool B>
__global__ void __launch_bounds__(kScopeThreads) scope_local_kernel(ScopeArgs a) { scope_local<B>(a); }
template <bool B>
__global__ void __launch_bounds__(kScopeThreads) scope_far_kernel(ScopeArgs a) { scope_far<B>(a); }
template <bool B>
__global__ void __launch_bounds__(kScopeThreads) scope_check_kernel(ScopeArgs a) { scope_check<B>(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_batch_sums_kernel(ScopeArgs a) { scope_batch_sums(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_batch_bases_kernel(ScopeArgs a) { scope_batch_bases(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_batch_starts_kernel(ScopeArgs a) { scope_batch_starts(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_batch_compact_kernel(ScopeArgs a) { scope_batch_compact(a); }
__global__ void __launch_bounds__(kScopeThreads) scope_batch_finish_kernel(ScopeArgs a) { scope_batch_finish(a); }

namespace {

constexpr uint32_t kFarGroups = 512;  // workgroups of the last kernel (4 waves each)

struct ScopeWs {
  int device;
  hipStream_t stream;
  void* mem;
  uint64_t bytes;
  uint64_t batch_cap;   // virtual entries a batch may hold (jsidx_scopes_reserve; 0: none)
  uint64_t batch_docs;  // documents a batch may hold
};
std::mutex g_smu;
std::vector<ScopeWs> g_sws;
constexpr uint64_t kBatchEntryLimit = (1ull << 31) - 1;  // levels stay below kNoLevel

// The scope workspace entry of (current device, stream), grown to `bytes`
// (synchronising the stream first); a failed growth removes the entry.
int scope_ws_entry(hipStream_t stream, uint64_t bytes, ScopeWs** out) {
  int dev = 0;
  *out = nullptr;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  for (size_t i = 0; i < g_sws.size(); i++) {
    ScopeWs& e = g_sws[i];
    if (e.device != dev || e.stream != stream) continue;
    if (e.bytes >= bytes) { *out = &e; return JSIDX_OK; }
    if (hipStreamSynchronize(stream) != hipSuccess) return JSIDX_E_HIP;
    (void)hipFree(e.mem);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      g_sws.erase(g_sws.begin() + (long)i);
      return JSIDX_E_NOWORKSPACE;
    }
    e.mem = p;
    e.bytes = bytes;
    *out = &e;
    return JSIDX_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return JSIDX_E_NOWORKSPACE;
  g_sws.push_back(ScopeWs{dev, stream, p, bytes, 0, 0});
  *out = &g_sws.back();
  return JSIDX_OK;
}

int scope_ws(hipStream_t stream, uint64_t bytes, void** out) {
  ScopeWs* e = nullptr;
  const int rc = scope_ws_entry(stream, bytes, &e);
  if (rc) return rc;
  *out = e->mem;
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
  (void)hipGetLastError();
  if (a.nchunks) hipLaunchKernelGGL(scope_chunk_fn_kernel<false>, dim3(a.nchunks), block, 0, stream, a);
  hipLaunchKernelGGL(scope_scan_kernel<false>, dim3(1), block, 0, stream, a);
  if (a.nchunks) {
    hipLaunchKernelGGL(scope_levels_kernel<false>, dim3(a.nchunks), block, 0, stream, a);
    hipLaunchKernelGGL(scope_local_kernel<false>, dim3(a.nchunks), block, 0, stream, a);
    hipLaunchKernelGGL(scope_far_kernel<false>, dim3(kFarGroups), block, 0, stream, a);
    hipLaunchKernelGGL(scope_check_kernel<false>, dim3(a.nchunks), block, 0, stream, a);
  }
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}

extern "C" int jsidx_scopes_reserve(uint64_t max_entries, uint32_t max_ndocs, jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (max_entries > kBatchEntryLimit) return JSIDX_E_TOO_LARGE;
  const uint64_t docs = max_ndocs ? max_ndocs : 1;
  const uint64_t single = scope_layout(max_entries).total, batch = scope_batch_layout(max_entries, docs).total;
  std::lock_guard<std::mutex> lk(g_smu);
  ScopeWs* e = nullptr;
  const int rc = scope_ws_entry(stream, single > batch ? single : batch, &e);
  if (rc) return rc;
  if (max_entries > e->batch_cap || docs > e->batch_docs) {
    e->batch_cap = max_entries;
    e->batch_docs = docs;
  }
  return JSIDX_OK;
}

extern "C" int jsidx_scopes_batch(const uint8_t* bufs, const uint64_t* offsets, uint32_t ndocs, const uint32_t* idx,
                                  const uint32_t* n, uint32_t* out_match, uint32_t* out_err,
                                  jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!bufs || !offsets || !idx || !n || !out_match || !out_err || ndocs == 0) return JSIDX_E_INVAL;
  std::lock_guard<std::mutex> lk(g_smu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  ScopeWs* e = nullptr;
  for (auto& w : g_sws)
    if (w.device == dev && w.stream == stream && w.batch_cap && w.batch_docs >= ndocs) e = &w;
  uint64_t cap = 0;
  if (e) {
    cap = e->batch_cap;
  } else {
    // no reservation for this batch: its entries are at most its bytes
    uint64_t ends[2] = {0, 0};
    if (hipMemcpyAsync(&ends[0], offsets, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(&ends[1], offsets + ndocs, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return JSIDX_E_HIP;
    cap = ends[1] > ends[0] ? ends[1] - ends[0] : 0;
    if (cap > kBatchEntryLimit) cap = kBatchEntryLimit;  // a larger batch is flagged on the device
    const int rc = scope_ws_entry(stream, scope_batch_layout(cap, ndocs).total, &e);
    if (rc) return rc;
  }
  const ScopeBatchLayout L = scope_batch_layout(cap, ndocs);
  uint8_t* m = static_cast<uint8_t*>(e->mem);
  ScopeArgs a;
  a.buf = bufs;
  a.len = 0;
  a.idx = idx;
  a.n = 0;
  a.nchunks = 0;
  a.match = reinterpret_cast<uint32_t*>(m + L.match);
  a.err = out_err;
  a.chunk_fn = reinterpret_cast<uint2*>(m + L.chunk_fn);
  a.in_depth = reinterpret_cast<uint2*>(m + L.in_depth);
  a.chunk_min = reinterpret_cast<uint32_t*>(m + L.chunk_min);
  a.qcount = reinterpret_cast<uint32_t*>(m + L.qcount);
  a.lev = reinterpret_cast<uint32_t*>(m + L.lev);
  a.queue = reinterpret_cast<uint32_t*>(m + L.queue);
  a.kind = m + L.kind;
  a.offsets = offsets;
  a.dn = n;
  a.ndocs = ndocs;
  a.cap = (uint32_t)cap;
  a.vn = reinterpret_cast<uint32_t*>(m + L.vn);
  a.part = reinterpret_cast<uint64_t*>(m + L.part);
  a.vstart = reinterpret_cast<uint32_t*>(m + L.vstart);
  a.docid = reinterpret_cast<uint32_t*>(m + L.docid);
  a.out_match = out_match;
  // grids for the reserved size; the kernels read the batch's own size on
  // the device and loop over its chunks and documents
  const uint64_t nch = (cap + kScopeChunk - 1) / kScopeChunk;
  const uint32_t chunk_groups = (uint32_t)(nch < 1 ? 1 : (nch < 2048 ? nch : 2048));
  const uint64_t dg = ((uint64_t)ndocs + kScopeThreads / kScopeWave - 1) / (kScopeThreads / kScopeWave);
  const uint32_t doc_groups = (uint32_t)(dg < 2048 ? dg : 2048);
  const dim3 block(kScopeThreads);
  (void)hipGetLastError();
  const dim3 sgrid((uint32_t)docscan_groups(ndocs));
  hipLaunchKernelGGL(scope_batch_sums_kernel, sgrid, block, 0, stream, a);
  hipLaunchKernelGGL(scope_batch_bases_kernel, dim3(1), block, 0, stream, a);
  hipLaunchKernelGGL(scope_batch_starts_kernel, sgrid, block, 0, stream, a);
  hipLaunchKernelGGL(scope_batch_compact_kernel, dim3(doc_groups), block, 0, stream, a);
  hipLaunchKernelGGL(scope_chunk_fn_kernel<true>, dim3(chunk_groups), block, 0, stream, a);
  hipLaunchKernelGGL(scope_scan_kernel<true>, dim3(1), block, 0, stream, a);
  hipLaunchKernelGGL(scope_levels_kernel<true>, dim3(chunk_groups), block, 0, stream, a);
  hipLaunchKernelGGL(scope_local_kernel<true>, dim3(chunk_groups), block, 0, stream, a);
  hipLaunchKernelGGL(scope_far_kernel<true>, dim3(kFarGroups), block, 0, stream, a);
  hipLaunchKernelGGL(scope_check_kernel<true>, dim3(chunk_groups), block, 0, stream, a);
  hipLaunchKernelGGL(scope_batch_finish_kernel, dim3(doc_groups), block, 0, stream, a);
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}
