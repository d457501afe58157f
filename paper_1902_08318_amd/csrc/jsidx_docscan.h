// jsidx_docscan.h -- the first virtual entry of each document of a batch: an
// exclusive scan of the documents' entry counts (an empty document may count
// one placeholder entry), in three passes so that no single workgroup walks
// all documents: per-group sums of 2048 documents, one workgroup scanning the
// group sums, and a per-group rescan that writes every document's start.
// Shared by the batched scope and tape kernels.
#pragma once
#include <stdint.h>

#include <jsidx_prims.h>  // resolved through the include path (the tests substitute their own)

namespace jsidx {

constexpr int kDScanThreads = 256;
constexpr int kDScanPer = 8;                              // documents per thread
constexpr int kDScanGroup = kDScanThreads * kDScanPer;    // documents per workgroup

struct DocScanLds {
  uint64_t s[kDScanThreads];
};

inline constexpr uint64_t docscan_groups(uint64_t ndocs) { return (ndocs + kDScanGroup - 1) / kDScanGroup; }

// Entries of document d.
JSIDX_DEV uint32_t docscan_count(const uint32_t* dn, uint64_t d, bool empty_as_one) {
  const uint32_t v = prim::load4(reinterpret_cast<const uint8_t*>(dn + d));
  return (v == 0u && empty_as_one) ? 1u : v;
}

// Inclusive scan of the workgroup's 256 values; returns the exclusive value
// and sets *all to the sum.
JSIDX_DEV uint64_t docscan_group(DocScanLds& g, uint32_t tid, uint64_t v, uint64_t* all) {
  g.s[tid] = v;
  prim::sync();
  for (uint32_t d = 1; d < (uint32_t)kDScanThreads; d <<= 1) {
    const uint64_t t = tid >= d ? g.s[tid - d] : 0u;
    prim::sync();
    g.s[tid] += t;
    prim::sync();
  }
  const uint64_t ex = g.s[tid] - v;
  *all = g.s[kDScanThreads - 1];
  prim::sync();
  return ex;
}

// Pass 1 (one workgroup per 2048 documents): the group's sum.
JSIDX_DEV void docscan_sums(const uint32_t* dn, uint32_t ndocs, bool empty_as_one, uint64_t* part) {
  DocScanLds& g = prim::lds_object<DocScanLds>();
  const uint32_t tid = prim::wave_id() * 64u + prim::lane();
  const uint64_t d0 = (uint64_t)prim::block() * kDScanGroup;
  uint64_t s = 0;
  for (int k = 0; k < kDScanPer; k++) {  // consecutive threads on consecutive documents
    const uint64_t d = d0 + (uint64_t)k * kDScanThreads + tid;
    if (d < ndocs) s += docscan_count(dn, d, empty_as_one);
  }
  uint64_t all = 0;
  (void)docscan_group(g, tid, s, &all);
  if (tid == 0) prim::st_pair(reinterpret_cast<uint2*>(part + prim::block()), (uint32_t)all, (uint32_t)(all >> 32));
}

// Pass 2 (one workgroup): the group sums become group bases; returns the
// total (every thread).
JSIDX_DEV uint64_t docscan_bases(uint32_t ngroups, uint64_t* part) {
  DocScanLds& g = prim::lds_object<DocScanLds>();
  const uint32_t tid = prim::wave_id() * 64u + prim::lane();
  const uint32_t per = (ngroups + kDScanThreads - 1) / kDScanThreads;
  const uint32_t lo = tid * per, hi = lo + per < ngroups ? lo + per : ngroups;
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; i++) {
    const uint2 v = prim::ld_pair(reinterpret_cast<const uint2*>(part + i));
    s += ((uint64_t)v.y << 32) | v.x;
  }
  uint64_t all = 0;
  uint64_t b = docscan_group(g, tid, s, &all);
  for (uint32_t i = lo; i < hi; i++) {
    const uint2 v = prim::ld_pair(reinterpret_cast<const uint2*>(part + i));
    prim::st_pair(reinterpret_cast<uint2*>(part + i), (uint32_t)b, (uint32_t)(b >> 32));
    b += ((uint64_t)v.y << 32) | v.x;
  }
  return all;
}

// Pass 3 (one workgroup per 2048 documents): each document's first virtual
// entry, given to fn(d, start, count) in turn (threads take runs of 8
// consecutive documents).
template <typename F>
JSIDX_DEV void docscan_starts(const uint32_t* dn, uint32_t ndocs, bool empty_as_one, const uint64_t* part, F fn) {
  DocScanLds& g = prim::lds_object<DocScanLds>();
  const uint32_t tid = prim::wave_id() * 64u + prim::lane();
  const uint64_t d0 = (uint64_t)prim::block() * kDScanGroup + (uint64_t)tid * kDScanPer;
  uint32_t c[kDScanPer];
  uint64_t s = 0;
  for (int k = 0; k < kDScanPer; k++) {
    c[k] = d0 + k < ndocs ? docscan_count(dn, d0 + k, empty_as_one) : 0u;
    s += c[k];
  }
  uint64_t all = 0;
  const uint2 pb = prim::ld_pair(reinterpret_cast<const uint2*>(part + prim::block()));
  uint64_t v = (((uint64_t)pb.y << 32) | pb.x) + docscan_group(g, tid, s, &all);
  for (int k = 0; k < kDScanPer; k++) {
    if (d0 + k >= ndocs) break;
    fn(d0 + k, v, c[k]);
    v += c[k];
  }
}

}  // namespace jsidx
