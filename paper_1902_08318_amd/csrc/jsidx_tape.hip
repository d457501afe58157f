// jsidx_tape.hip -- the stage-2 tape (Sec. 3, Fig. 2) behind jsidx_tape of
// include/jsidx.h.  The kernel bodies and the method are in jsidx_tape.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "jsidx.h"
#include "jsidx_tape.h"

namespace jsidx {

// one document: registers kept to five waves per SIMD (the batch form
// needs more)
template <bool B>
__global__ void __launch_bounds__(kTapeThreads) tape_count_kernel(TapeArgs a);
template <>
__global__ void __launch_bounds__(kTapeThreads) __attribute__((amdgpu_waves_per_eu(5)))
tape_count_kernel<false>(TapeArgs a) { tape_count<false>(a); }
template <>
__global__ void __launch_bounds__(kTapeThreads) tape_count_kernel<true>(TapeArgs a) { tape_count<true>(a); }
template <bool B>
__global__ void __launch_bounds__(kTapeThreads) tape_scan_kernel(TapeArgs a) { tape_scan<B>(a); }
template <bool B>
__global__ void __launch_bounds__(kTapeThreads) tape_offsets_kernel(TapeArgs a) { tape_offsets<B>(a); }
// four workgroups per CU fit its LDS: registers are kept to that occupancy too
template <bool B>
__global__ void __launch_bounds__(kTapeThreads) __attribute__((amdgpu_waves_per_eu(4))) tape_write_kernel(TapeArgs a) {
  tape_write<B>(a);
}
// a thread per atom waits mostly on its window: registers kept to eight
// waves per SIMD (64, no spills) to have more atoms in flight
template <bool B>
__global__ void __launch_bounds__(kTapeThreads) __attribute__((amdgpu_waves_per_eu(8))) tape_numbers_kernel(TapeArgs a) {
  tape_numbers<B>(a);
}
template <bool B>
__global__ void __launch_bounds__(kExactThreads) tape_exact_kernel(TapeArgs a) { tape_exact<B>(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_batch_sums_kernel(TapeArgs a) { tape_batch_sums(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_batch_bases_kernel(TapeArgs a) { tape_batch_bases(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_batch_starts_kernel(TapeArgs a) { tape_batch_starts(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_batch_compact_kernel(TapeArgs a) { tape_batch_compact(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_batch_docs_kernel(TapeArgs a) { tape_batch_docs(a); }

namespace {

struct TapeWs {
  int device;
  hipStream_t stream;
  void* mem;
  uint64_t bytes;
  uint64_t batch_cap;   // virtual entries a batch may hold (jsidx_tape_reserve; 0: none)
  uint64_t batch_docs;  // documents a batch may hold
};
std::mutex g_tmu;
std::vector<TapeWs> g_tws;

// The tape workspace entry of (current device, stream), grown to `bytes`
// (synchronising the stream first); a failed growth removes the entry.
int tape_ws_entry(hipStream_t stream, uint64_t bytes, TapeWs** out) {
  int dev = 0;
  *out = nullptr;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  for (size_t i = 0; i < g_tws.size(); i++) {
    TapeWs& e = g_tws[i];
    if (e.device != dev || e.stream != stream) continue;
    if (e.bytes >= bytes) { *out = &e; return JSIDX_OK; }
    if (hipStreamSynchronize(stream) != hipSuccess) return JSIDX_E_HIP;
    (void)hipFree(e.mem);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      g_tws.erase(g_tws.begin() + (long)i);
      return JSIDX_E_NOWORKSPACE;
    }
    e.mem = p;
    e.bytes = bytes;
    *out = &e;
    return JSIDX_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return JSIDX_E_NOWORKSPACE;
  g_tws.push_back(TapeWs{dev, stream, p, bytes, 0, 0});
  *out = &g_tws.back();
  return JSIDX_OK;
}

int tape_ws(hipStream_t stream, uint64_t bytes, void** out) {
  TapeWs* e = nullptr;
  const int rc = tape_ws_entry(stream, bytes, &e);
  if (rc) return rc;
  *out = e->mem;
  return JSIDX_OK;
}

}  // namespace
}  // namespace jsidx

using namespace jsidx;

extern "C" int jsidx_tape(const uint8_t* buf, uint64_t len, const uint32_t* idx, uint32_t n, const uint32_t* match,
                          uint64_t* out_tape, uint64_t* out_tape_n, uint8_t* out_str, uint64_t* out_str_n,
                          uint32_t* out_err, jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!out_tape || !out_tape_n || !out_str_n || !out_err) return JSIDX_E_INVAL;
  if (n && (!buf || !idx || !match || !out_str)) return JSIDX_E_INVAL;
  if (len >= (1ull << 32) - (1ull << 16) || n >= (1u << 31)) return JSIDX_E_INVAL;
  const TapeLayout L = tape_layout(n);
  std::lock_guard<std::mutex> lk(g_tmu);
  void* mem = nullptr;
  int rc = tape_ws(stream, L.total, &mem);
  if (rc) return rc;
  uint8_t* m = static_cast<uint8_t*>(mem);
  TapeArgs a;
  a.buf = buf ? buf : reinterpret_cast<const uint8_t*>(out_err);  // never read when n == 0
  a.len = len;
  a.idx = idx;
  a.n = n;
  a.nchunks = (uint32_t)((n + (uint64_t)kTapeChunk - 1) / kTapeChunk);
  a.match = match;
  a.tape = out_tape;
  a.str = out_str ? out_str : reinterpret_cast<uint8_t*>(out_err);  // never written when n == 0
  a.tape_n = out_tape_n;
  a.str_n = out_str_n;
  a.err = out_err;
  a.chunk_sum = reinterpret_cast<uint64_t*>(m + L.chunk_sum);
  a.sbytes = reinterpret_cast<uint32_t*>(m + L.sbytes);
  a.toff = reinterpret_cast<uint32_t*>(m + L.toff);
  a.kb = m + L.kb;
  a.runbad = m + L.runbad;
  a.qcount = reinterpret_cast<uint32_t*>(m + L.qcount);
  a.queue = reinterpret_cast<uint32_t*>(m + L.queue);
  a.nqueue = reinterpret_cast<uint2*>(m + L.nqueue);
  const dim3 block(kTapeThreads);
  (void)hipGetLastError();
  if (a.nchunks) hipLaunchKernelGGL(tape_count_kernel<false>, dim3(a.nchunks), block, 0, stream, a);
  hipLaunchKernelGGL(tape_scan_kernel<false>, dim3(1), block, 0, stream, a);
  if (a.nchunks) {
    hipLaunchKernelGGL(tape_offsets_kernel<false>, dim3(a.nchunks), block, 0, stream, a);
    hipLaunchKernelGGL(tape_write_kernel<false>, dim3(a.nchunks), block, 0, stream, a);
    // the number queue holds at most n entries; a grid-stride loop takes the rest
    const uint64_t qgroups = ((uint64_t)n + kTapeThreads - 1) / kTapeThreads;
    const dim3 qgrid((uint32_t)(qgroups < kQueueGroups ? qgroups : kQueueGroups));
    hipLaunchKernelGGL(tape_numbers_kernel<false>, qgrid, block, 0, stream, a);
    hipLaunchKernelGGL(tape_exact_kernel<false>, dim3(kExactGroups), dim3(kExactThreads), 0, stream, a);
  }
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}

extern "C" int jsidx_tape_reserve(uint64_t max_entries, uint32_t max_ndocs, jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (max_entries >= (1ull << 31)) return JSIDX_E_TOO_LARGE;
  const uint64_t docs = max_ndocs ? max_ndocs : 1;
  const uint64_t single = tape_layout(max_entries).total, batch = tape_batch_layout(max_entries + docs, docs).total;
  std::lock_guard<std::mutex> lk(g_tmu);
  TapeWs* e = nullptr;
  const int rc = tape_ws_entry(stream, single > batch ? single : batch, &e);
  if (rc) return rc;
  if (max_entries + docs > e->batch_cap || docs > e->batch_docs) {
    e->batch_cap = max_entries + docs;  // an empty document takes one placeholder entry
    e->batch_docs = docs;
  }
  return JSIDX_OK;
}

extern "C" int jsidx_tape_batch(const uint8_t* bufs, const uint64_t* offsets, uint32_t ndocs, const uint32_t* idx,
                                const uint32_t* n, const uint32_t* match, uint64_t* out_tape, uint64_t tape_cap,
                                uint8_t* out_str, uint64_t str_cap, uint64_t* out_pos, uint32_t* out_err,
                                jsidx_stream_t stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!bufs || !offsets || !idx || !n || !match || !out_tape || !out_str || !out_pos || !out_err || ndocs == 0)
    return JSIDX_E_INVAL;
  std::lock_guard<std::mutex> lk(g_tmu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  TapeWs* e = nullptr;
  for (auto& w : g_tws)
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
    cap = (ends[1] > ends[0] ? ends[1] - ends[0] : 0) + ndocs;
    if (cap >= (1ull << 31)) cap = (1ull << 31) - 1;  // a larger batch is flagged on the device
    const int rc = tape_ws_entry(stream, tape_batch_layout(cap, ndocs).total, &e);
    if (rc) return rc;
  }
  const TapeBatchLayout L = tape_batch_layout(cap, ndocs);
  uint8_t* m = static_cast<uint8_t*>(e->mem);
  TapeArgs a;
  a.buf = bufs;
  a.len = 0;
  a.idx = idx;
  a.n = 0;
  a.nchunks = 0;
  a.match = match;
  a.tape = out_tape;
  a.str = out_str;
  a.tape_n = nullptr;
  a.str_n = nullptr;
  a.err = out_err;
  a.chunk_sum = reinterpret_cast<uint64_t*>(m + L.chunk_sum);
  a.sbytes = reinterpret_cast<uint32_t*>(m + L.sbytes);
  a.toff = reinterpret_cast<uint32_t*>(m + L.toff);
  a.kb = m + L.kb;
  a.runbad = m + L.runbad;
  a.qcount = reinterpret_cast<uint32_t*>(m + L.qcount);
  a.queue = reinterpret_cast<uint32_t*>(m + L.queue);
  a.nqueue = reinterpret_cast<uint2*>(m + L.nqueue);
  a.offsets = offsets;
  a.dn = n;
  a.ndocs = ndocs;
  a.cap = (uint32_t)cap;
  a.tape_cap = tape_cap;
  a.str_cap = str_cap;
  a.vn = reinterpret_cast<uint32_t*>(m + L.vn);
  a.tot = reinterpret_cast<uint64_t*>(m + L.tot);
  a.part = reinterpret_cast<uint64_t*>(m + L.part);
  a.vstart = reinterpret_cast<uint32_t*>(m + L.vstart);
  a.docid = reinterpret_cast<uint32_t*>(m + L.docid);
  a.vpos = reinterpret_cast<uint64_t*>(m + L.vpos);
  a.vflag = m + L.vflag;
  a.dbase = reinterpret_cast<uint64_t*>(m + L.dbase);
  a.out_pos = out_pos;
  // grids for the reserved size; the kernels read the batch's own size on
  // the device and loop over its chunks, documents and queues
  const uint64_t nch = (cap + kTapeChunk - 1) / kTapeChunk;
  const uint32_t chunk_groups = (uint32_t)(nch < 1 ? 1 : (nch < 4096 ? nch : 4096));
  const uint64_t dg = ((uint64_t)ndocs + 3) / 4;
  const uint32_t doc_groups = (uint32_t)(dg < 2048 ? dg : 2048);
  const uint64_t qgroups = (cap + kTapeThreads - 1) / kTapeThreads;
  const dim3 qgrid((uint32_t)(qgroups < kQueueGroups ? qgroups : kQueueGroups));
  const dim3 block(kTapeThreads);
  (void)hipGetLastError();
  const dim3 sgrid((uint32_t)docscan_groups(ndocs));
  hipLaunchKernelGGL(tape_batch_sums_kernel, sgrid, block, 0, stream, a);
  hipLaunchKernelGGL(tape_batch_bases_kernel, dim3(1), block, 0, stream, a);
  hipLaunchKernelGGL(tape_batch_starts_kernel, sgrid, block, 0, stream, a);
  hipLaunchKernelGGL(tape_batch_compact_kernel, dim3(doc_groups), block, 0, stream, a);
  hipLaunchKernelGGL(tape_count_kernel<true>, dim3(chunk_groups), block, 0, stream, a);
  hipLaunchKernelGGL(tape_scan_kernel<true>, dim3(1), block, 0, stream, a);
  hipLaunchKernelGGL(tape_offsets_kernel<true>, dim3(chunk_groups), block, 0, stream, a);
  hipLaunchKernelGGL(tape_batch_docs_kernel, dim3((ndocs + kTapeThreads - 1) / kTapeThreads), block, 0, stream, a);
  hipLaunchKernelGGL(tape_write_kernel<true>, dim3(chunk_groups), block, 0, stream, a);
  hipLaunchKernelGGL(tape_numbers_kernel<true>, qgrid, block, 0, stream, a);
  hipLaunchKernelGGL(tape_exact_kernel<true>, dim3(kExactGroups), dim3(kExactThreads), 0, stream, a);
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}
