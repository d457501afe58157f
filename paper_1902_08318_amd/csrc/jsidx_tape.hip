// jsidx_tape.hip -- the stage-2 tape (Sec. 3, Fig. 2) behind jsidx_tape of
// include/jsidx.h.  The kernel bodies and the method are in jsidx_tape.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "jsidx.h"
#include "jsidx_tape.h"

namespace jsidx {

__global__ void __launch_bounds__(kTapeThreads) tape_count_kernel(TapeArgs a) { tape_count(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_scan_kernel(TapeArgs a) { tape_scan(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_offsets_kernel(TapeArgs a) { tape_offsets(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_write_kernel(TapeArgs a) { tape_write(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_strings_kernel(TapeArgs a) { tape_strings(a); }
__global__ void __launch_bounds__(kTapeThreads) tape_numbers_kernel(TapeArgs a) { tape_numbers(a); }
__global__ void __launch_bounds__(kExactThreads) tape_exact_kernel(TapeArgs a) { tape_exact(a); }

namespace {

struct TapeWs {
  int device;
  hipStream_t stream;
  void* mem;
  uint64_t bytes;
};
std::mutex g_tmu;
std::vector<TapeWs> g_tws;

// The tape workspace of (current device, stream), grown to `bytes`.
int tape_ws(hipStream_t stream, uint64_t bytes, void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return JSIDX_E_HIP;
  for (auto& e : g_tws) {
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
  g_tws.push_back(TapeWs{dev, stream, p, bytes});
  *out = p;
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
  a.qcount = reinterpret_cast<uint32_t*>(m + L.qcount);
  a.queue = reinterpret_cast<uint32_t*>(m + L.queue);
  a.squeue = reinterpret_cast<uint64_t*>(m + L.squeue);
  a.nqueue = reinterpret_cast<uint32_t*>(m + L.nqueue);
  const dim3 block(kTapeThreads);
  if (a.nchunks) hipLaunchKernelGGL(tape_count_kernel, dim3(a.nchunks), block, 0, stream, a);
  hipLaunchKernelGGL(tape_scan_kernel, dim3(1), block, 0, stream, a);
  if (a.nchunks) {
    hipLaunchKernelGGL(tape_offsets_kernel, dim3(a.nchunks), block, 0, stream, a);
    hipLaunchKernelGGL(tape_write_kernel, dim3(a.nchunks), block, 0, stream, a);
    // the queues hold at most n entries; a grid-stride loop takes the rest
    const uint64_t qgroups = ((uint64_t)n + kTapeThreads - 1) / kTapeThreads;
    const dim3 qgrid((uint32_t)(qgroups < kQueueGroups ? qgroups : kQueueGroups));
    hipLaunchKernelGGL(tape_strings_kernel, qgrid, block, 0, stream, a);
    hipLaunchKernelGGL(tape_numbers_kernel, qgrid, block, 0, stream, a);
    hipLaunchKernelGGL(tape_exact_kernel, dim3(kExactGroups), dim3(kExactThreads), 0, stream, a);
  }
  if (hipGetLastError() != hipSuccess) return JSIDX_E_HIP;
  return JSIDX_OK;
}
