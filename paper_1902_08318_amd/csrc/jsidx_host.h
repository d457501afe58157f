// jsidx_host.h -- host-side pieces of the indexing library shared by its
// source files: a workspace and the launch over it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "jsidx_kernel.h"

namespace jsidx {

// A launch's workspace: device memory of cap_tiles largest tiles.
struct StreamWs {
  int device;
  hipStream_t stream;
  Workspace* ws;
  uint64_t cap_tiles;  // in largest tiles
  bool reserved;  // sized by jsidx_reserve: batch calls trust it and never sync
  uint64_t doc_off;  // byte offset of the one-document kernel's region from ws
};

// Guards the library's host state (workspaces, tuning table, variant).
extern std::mutex g_mu;

// Launches the indexing (or minify) kernel over workspace e.  span >= 0: the
// bytes from the 16-byte granule holding the first byte to the end (one
// document); span < 0: a batch (sizes on the device).  Caller holds g_mu.
int launch(Args& a, hipStream_t stream, const StreamWs& e, int64_t span, bool minify);

// Launches the one-document kernel (jsidx_doc.h) over workspace e.  Caller
// holds g_mu.
int launch_doc(const uint8_t* buf, uint64_t len, uint32_t* out, uint32_t* out_n, uint32_t* out_err,
               hipStream_t stream, const StreamWs& e);

}  // namespace jsidx
