// jsidx_scopes.h -- scope matching over a document's structural index, the
// scope links of the paper's tape (Sec. 3, Fig. 2: the start of an object or
// array is linked to its end and back).  Written on the same primitives as
// the indexing kernel (jsidx_prims.h), so that the CPU emulation of the tests
// runs this source too.
//
// The reference semantics are those of a bracket stack over the index
// entries: an opening bracket is pushed, a closing one is linked with the top
// of the stack (MISMATCHED if the kinds differ) or, with the stack empty, left
// unlinked (UNBALANCED), and openers left at the end are unlinked
// (UNBALANCED).  In parallel:
//   1. Each entry is a function of the depth before it: an opener adds one, a
//      closer subtracts one but not below zero (an unmatched closer leaves the
//      depth at 0), x -> max(x + a, b); these compose, so per chunk of 4096
//      entries the composed function is computed (scope_chunk_fn) and a scan
//      over the chunks gives the depth entering each chunk (scope_scan).
//   2. Each bracket gets its level: an opener the depth before it, a linked
//      closer the depth after it (scope_levels).  A stack links an opener at
//      level L with the first later entry whose level is at most L, which is
//      the closer that returns the depth to L.
//   3. That entry is searched in the opener's chunk, in LDS (scope_local), and
//      for scopes that leave their chunk, over the chunks' minimum levels and
//      then inside the first chunk that can hold it, 64 entries per step by a
//      whole wave (scope_far).
//   4. With the links known, a per-entry pass checks that the tokens form one
//      JSON value (scope_check, below).
#pragma once

#include "jsidx_device.h"
#include "jsidx_docscan.h"

namespace jsidx {

constexpr int kScopeWave = 64;      // lanes per wave
constexpr int kScopeThreads = 256;  // four waves per workgroup
constexpr int kScopePer = 16;       // entries per thread
constexpr int kScopeChunk = kScopeThreads * kScopePer;
constexpr uint32_t kNoLevel = 0xFFFFFFFFu;
constexpr uint32_t kUnlinked = 0xFFFFFFFFu;
constexpr uint32_t kErrUnbalanced = 0x10u;
constexpr uint32_t kErrMismatched = 0x20u;
constexpr uint32_t kErrSyntax = 0x40u;
// Token of an index entry, by its byte: atoms (numbers, literals, anything
// else) are kOther, a string is its opening quote.  In the workspace's kind
// array bit 3 (kRootBit) marks entries at depth 0 and bit 4 (kMemberBit) a
// linked closer whose opener follows a colon (the scope is a member's value).
enum : uint32_t { kOther = 0, kOpenSq = 1, kOpenCu = 2, kCloseSq = 3, kCloseCu = 4, kColon = 5, kComma = 6, kStr = 7 };
constexpr uint32_t kTokMask = 7u;
constexpr uint32_t kRootBit = 8u;
constexpr uint32_t kMemberBit = 16u;

struct DepthFn {  // x -> max(x + a, b)
  int64_t a, b;
};
constexpr int64_t kNegInf = -(1ll << 62);

JSIDX_DEV DepthFn fn_id() { return DepthFn{0, kNegInf}; }
JSIDX_DEV DepthFn fn_then(const DepthFn& f, const DepthFn& g) {  // f, then g
  // terms stay in [kNegInf, 2^32), so one sum cannot overflow; clamping at
  // kNegInf keeps it so through any number of resets (batches)
  const int64_t a = f.a + g.a, fb = f.b + g.a;
  const int64_t b = fb > g.b ? fb : g.b;
  return DepthFn{a < kNegInf ? kNegInf : a, b < kNegInf ? kNegInf : b};
}
JSIDX_DEV int64_t fn_apply(const DepthFn& f, int64_t x) { return x + f.a > f.b ? x + f.a : f.b; }
JSIDX_DEV DepthFn fn_of(uint32_t kind) {
  if (kind == kOpenSq || kind == kOpenCu) return DepthFn{1, kNegInf};
  if (kind == kCloseSq || kind == kCloseCu) return DepthFn{-1, 0};
  return fn_id();
}

struct ScopeArgs {
  const uint8_t* buf;
  uint64_t len;
  const uint32_t* idx;
  uint32_t n;
  uint32_t nchunks;
  uint32_t* match;
  uint32_t* err;
  // workspace
  uint2* chunk_fn;      // 2 per chunk: a, b
  uint2* in_depth;      // per chunk
  uint32_t* chunk_min;  // per chunk: lowest level
  uint32_t* qcount;     // scopes that leave their chunk
  uint32_t* lev;        // per entry: level of a bracket (kNoLevel otherwise)
  uint8_t* kind;        // per entry: token (an unmatched closer becomes
                        // kOther), kRootBit if the depth before it is 0
  uint32_t* queue;      // per entry at most
  // batches (jsidx_scopes_batch): the documents' entries laid end to end as
  // one sequence of "virtual" entries; n and nchunks then live on the device
  const uint64_t* offsets;  // ndocs + 1 byte offsets of the documents in buf
  const uint32_t* dn;       // per document: its entry count (idx holds them at idx + offsets[d])
  uint32_t ndocs;
  uint32_t cap;             // virtual entries the workspace holds
  uint32_t* vn;             // [0] virtual entries, [1] their chunks, [2] 1 if the batch is over
                            // capacity (set by scope_batch_bases)
  uint64_t* part;           // per 2048 documents: entry sum, then base
  uint32_t* vstart;         // ndocs + 1: first virtual entry of each document
  uint32_t* docid;          // per virtual entry: its document
  uint32_t* out_match;      // batch layout, like idx
};

// Kind-array bits of batches: the first and last entry of a document.
constexpr uint32_t kDocStartBit = 32u;
constexpr uint32_t kDocEndBit = 64u;
// x -> 0: the depth at a document's first entry (the composition then adds
// the entry's own step).
JSIDX_DEV DepthFn fn_reset() { return DepthFn{kNegInf, 0}; }

// Workspace layout for n entries (byte offsets; host side).
struct ScopeLayout {
  uint64_t chunk_fn, in_depth, chunk_min, qcount, lev, queue, kind, total;
};
inline uint64_t scope_align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }
inline ScopeLayout scope_layout(uint64_t n) {
  const uint64_t nc = (n + kScopeChunk - 1) / kScopeChunk;
  ScopeLayout L;
  uint64_t o = 0;
  L.chunk_fn = o; o = scope_align256(o + nc * 16);
  L.in_depth = o; o = scope_align256(o + nc * 8);
  L.chunk_min = o; o = scope_align256(o + nc * 4);
  L.qcount = o; o = scope_align256(o + 4);
  L.lev = o; o = scope_align256(o + n * 4);
  L.queue = o; o = scope_align256(o + n * 4);
  L.kind = o; o = scope_align256(o + n);
  L.total = o;
  return L;
}

// Workspace layout of a batch of up to cap virtual entries in up to maxdocs
// documents (byte offsets; host side).
struct ScopeBatchLayout {
  uint64_t vn, qcount, part, vstart, docid, chunk_fn, in_depth, chunk_min, lev, queue, match, kind, total;
};
inline ScopeBatchLayout scope_batch_layout(uint64_t cap, uint64_t maxdocs) {
  const uint64_t nc = (cap + kScopeChunk - 1) / kScopeChunk;
  ScopeBatchLayout L;
  uint64_t o = 0;
  L.vn = o; o = scope_align256(o + 8);
  L.qcount = o; o = scope_align256(o + 4);
  L.part = o; o = scope_align256(o + (docscan_groups(maxdocs) + 1) * 8);
  L.vstart = o; o = scope_align256(o + (maxdocs + 1) * 4);
  L.docid = o; o = scope_align256(o + cap * 4);
  L.chunk_fn = o; o = scope_align256(o + nc * 16);
  L.in_depth = o; o = scope_align256(o + nc * 8);
  L.chunk_min = o; o = scope_align256(o + nc * 4);
  L.lev = o; o = scope_align256(o + cap * 4);
  L.queue = o; o = scope_align256(o + cap * 4);
  L.match = o; o = scope_align256(o + cap * 4);
  L.kind = o; o = scope_align256(o + cap);
  L.total = o;
  return L;
}

JSIDX_DEV uint2 pack64(int64_t v) {
  uint2 r;
  r.x = (uint32_t)(uint64_t)v;
  r.y = (uint32_t)((uint64_t)v >> 32);
  return r;
}
JSIDX_DEV int64_t unpack64(uint2 v) { return (int64_t)(((uint64_t)v.y << 32) | v.x); }

JSIDX_DEV uint32_t kind_of_byte(uint32_t b) {
  return b == 0x5Bu ? kOpenSq : b == 0x7Bu ? kOpenCu : b == 0x5Du ? kCloseSq : b == 0x7Du ? kCloseCu
       : b == 0x3Au ? kColon : b == 0x2Cu ? kComma : b == 0x22u ? kStr : kOther;
}

// LDS of the kernels: each takes only what it uses, so that more workgroups
// fit on a CU.
constexpr int kScopeRunGroup = 16;  // runs per group of run minima (scope_local)
struct ScopeGroup {
  DepthFn f[kScopeThreads];
  uint32_t m[kScopeThreads];
  uint32_t m2[kScopeThreads / kScopeRunGroup];  // lowest level of each group of runs
  uint32_t L[kScopeChunk];  // levels of the chunk's entries
  alignas(4) uint8_t K[kScopeChunk];  // kinds of the chunk's entries
};
struct ScopeFold {
  DepthFn f[kScopeThreads];
  alignas(4) uint8_t K[kScopeChunk];
};
struct ScopeScanLds {
  DepthFn f[kScopeThreads];
};
constexpr int kCheckWords = (kScopeChunk + 8) / 4;
struct ScopeCheckLds {
  uint32_t W[kCheckWords];  // kind bytes of entries c0 - 4 .. c0 + kScopeChunk + 3
};

JSIDX_DEV uint32_t scope_tid() { return prim::wave_id() * kScopeWave + prim::lane(); }

// Entries and chunks of the launch: the arguments for one document, the
// device for a batch (scope_batch_bases wrote them).
template <bool BATCH>
JSIDX_DEV uint32_t n_of(const ScopeArgs& a) { return BATCH ? prim::ld_agent32(a.vn) : a.n; }
template <bool BATCH>
JSIDX_DEV uint32_t nchunks_of(const ScopeArgs& a) { return BATCH ? prim::ld_agent32(a.vn + 1) : a.nchunks; }
// The flags word an error of virtual entry i goes to.
template <bool BATCH>
JSIDX_DEV uint32_t* err_of(const ScopeArgs& a, uint64_t i) {
  return BATCH ? a.err + prim::load4(reinterpret_cast<const uint8_t*>(a.docid + i)) : a.err;
}
// An entry's step of the depth: at a document's first entry (batches) the
// depth starts again from 0.
JSIDX_DEV DepthFn fn_of_entry(uint32_t kb) {
  const DepthFn f = fn_of(kb & kTokMask);
  return (kb & kDocStartBit) ? fn_then(fn_reset(), f) : f;
}

// The kinds of chunk c's entries into LDS: consecutive threads read
// consecutive entries (coalesced), then each thread works on its own run of
// kScopePer entries in LDS.
template <typename G>
JSIDX_DEV void load_kinds(const ScopeArgs& a, G& g, uint32_t tid, uint32_t c) {
  const uint64_t c0 = (uint64_t)c * kScopeChunk;
  constexpr int kR = kScopeChunk / kScopeThreads;
  // all positions, then all bytes, in flight together (a position outside
  // the document, and an entry past n, is kOther)
  uint32_t p[kR], b[kR];
#pragma unroll
  for (int k = 0; k < kR; k++) {
    const uint64_t i = c0 + tid + (uint64_t)k * kScopeThreads;
    p[k] = i < a.n ? prim::load4(reinterpret_cast<const uint8_t*>(a.idx + i)) : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int k = 0; k < kR; k++) b[k] = (uint64_t)p[k] < a.len ? prim::load1(a.buf + p[k]) : 0u;
#pragma unroll
  for (int k = 0; k < kR; k++) g.K[tid + (uint32_t)k * kScopeThreads] = (uint8_t)kind_of_byte(b[k]);
  prim::sync();
}

// The same from the kind array (written by scope_chunk_fn, or for a batch by
// scope_batch_compact; one word per thread and step; entries past n read as
// kOther).
template <typename G>
JSIDX_DEV void load_stored_kinds(const ScopeArgs& a, uint32_t n, G& g, uint32_t tid, uint32_t c) {
  const uint64_t c0 = (uint64_t)c * kScopeChunk;
  uint32_t* kw = reinterpret_cast<uint32_t*>(g.K);
  for (uint32_t w = tid; w < (uint32_t)kScopeChunk / 4; w += kScopeThreads) {
    const uint64_t b = c0 + 4 * (uint64_t)w;
    uint32_t v = 0u;  // four kOther
    if (b < n) {
      v = prim::load4(a.kind + b);
      const uint64_t valid = n - b;
      if (valid < 4) v &= ~(0xFFFFFFFFu << (8 * valid));
    }
    kw[w] = v;
  }
  prim::sync();
}

// A lane's function from the lane d below it (shuffled as four words).
JSIDX_DEV DepthFn fn_shfl_up(const DepthFn& f, int d) {
  const uint64_t a = (uint64_t)f.a, b = (uint64_t)f.b;
  const uint64_t ua = ((uint64_t)prim::shfl_up((uint32_t)(a >> 32), d) << 32) | prim::shfl_up((uint32_t)a, d);
  const uint64_t ub = ((uint64_t)prim::shfl_up((uint32_t)(b >> 32), d) << 32) | prim::shfl_up((uint32_t)b, d);
  return DepthFn{(int64_t)ua, (int64_t)ub};
}

// Ordered exclusive scan of the workgroup's per-thread functions: each wave
// scans its lanes by shuffles, then the four wave totals are composed in
// order (two barriers); returns the composition of the threads before this
// one.
template <typename G>
JSIDX_DEV DepthFn group_exclusive(G& g, uint32_t tid, DepthFn mine) {
  static_assert(kScopeThreads == 4 * kScopeWave, "four waves");
  const uint32_t lane = tid % (uint32_t)kScopeWave, wv = tid / (uint32_t)kScopeWave;
  DepthFn incl = mine;
#pragma unroll
  for (int d = 1; d < kScopeWave; d <<= 1) {
    const DepthFn up = fn_shfl_up(incl, d);
    if (lane >= (uint32_t)d) incl = fn_then(up, incl);
  }
  const DepthFn up1 = fn_shfl_up(incl, 1);
  if (lane == (uint32_t)kScopeWave - 1) g.f[wv] = incl;
  prim::sync();
  DepthFn ex = fn_id();
  for (uint32_t k = 0; k < wv; k++) ex = fn_then(ex, g.f[k]);
  if (lane) ex = fn_then(ex, up1);
  prim::sync();
  return ex;
}

// 1. The composed depth function of each chunk (one workgroup per chunk).
template <bool BATCH>
JSIDX_DEVFN void scope_chunk_fn(const ScopeArgs& a) {
  ScopeFold& g = prim::lds_object<ScopeFold>();
  const uint32_t tid = scope_tid();
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  if (BATCH) {
    load_stored_kinds(a, n, g, tid, c);
  } else {
    load_kinds(a, g, tid, c);
    // the kinds go to the workspace as words, for the kernels after this one
    // (the word holding entry n - 1 lies inside the array's 256-byte padding)
    const uint64_t c0 = (uint64_t)c * kScopeChunk;
    const uint32_t* kw = reinterpret_cast<const uint32_t*>(g.K);
    for (uint32_t w = tid; w < (uint32_t)kScopeChunk / 4; w += kScopeThreads) {
      if (c0 + 4 * (uint64_t)w >= a.n) break;
      prim::st_out(reinterpret_cast<uint32_t*>(a.kind + c0) + w, kw[w]);
    }
  }
  DepthFn f = fn_id();
  for (int k = 0; k < kScopePer; k++) f = fn_then(f, fn_of_entry(g.K[tid * kScopePer + k]));
  const DepthFn ex = group_exclusive(g, tid, f);
  if (tid == kScopeThreads - 1) {
    const DepthFn all = fn_then(ex, f);
    prim::st_pair(a.chunk_fn + 2 * (uint64_t)c, pack64(all.a).x, pack64(all.a).y);
    prim::st_pair(a.chunk_fn + 2 * (uint64_t)c + 1, pack64(all.b).x, pack64(all.b).y);
  }
  prim::sync();
  }
}

// 2. The depth entering each chunk (one workgroup); for one document also
//    clears the flags and the queue for the kernels after it (for a batch,
//    scope_batch_bases and scope_batch_starts did).
template <bool BATCH>
JSIDX_DEVFN void scope_scan(const ScopeArgs& a) {
  ScopeScanLds& g = prim::lds_object<ScopeScanLds>();
  const uint32_t tid = scope_tid();
  const uint32_t nchunks = nchunks_of<BATCH>(a);
  const uint32_t per = (nchunks + kScopeThreads - 1) / kScopeThreads;
  const uint64_t lo = (uint64_t)tid * per;
  const uint64_t hi = lo + per < nchunks ? lo + per : nchunks;
  // each thread's run of chunks, eight loads in flight at a time
  constexpr int kB = 8;
  DepthFn f = fn_id();
  for (uint64_t c = lo; c < hi; c += kB) {
    DepthFn fc[kB];
#pragma unroll
    for (int k = 0; k < kB; k++)
      fc[k] = c + k < hi ? DepthFn{unpack64(prim::ld_pair(a.chunk_fn + 2 * (c + k))),
                                   unpack64(prim::ld_pair(a.chunk_fn + 2 * (c + k) + 1))}
                         : fn_id();
#pragma unroll
    for (int k = 0; k < kB; k++) f = fn_then(f, fc[k]);
  }
  const DepthFn ex = group_exclusive(g, tid, f);
  int64_t x = fn_apply(ex, 0);
  for (uint64_t c = lo; c < hi; c += kB) {
    DepthFn fc[kB];
#pragma unroll
    for (int k = 0; k < kB; k++)
      fc[k] = c + k < hi ? DepthFn{unpack64(prim::ld_pair(a.chunk_fn + 2 * (c + k))),
                                   unpack64(prim::ld_pair(a.chunk_fn + 2 * (c + k) + 1))}
                         : fn_id();
#pragma unroll
    for (int k = 0; k < kB; k++) {
      if (c + k < hi) prim::st_pair(a.in_depth + c + k, pack64(x).x, pack64(x).y);
      x = fn_apply(fc[k], x);
    }
  }
  if (!BATCH && tid == 0) {
    prim::st_out(a.err, a.n ? 0u : kErrSyntax);  // an empty index holds no value
    prim::st_out(a.qcount, 0u);
  }
}

// 3. Levels and kinds of the entries, the lowest level of each chunk, and
//    every link cleared (one workgroup per chunk).  In a batch a level is
//    offset by the first virtual entry of its document, which is more than
//    any level of an earlier document, so no search ever crosses into
//    another document.
template <bool BATCH>
JSIDX_DEVFN void scope_levels(const ScopeArgs& a) {
  ScopeGroup& g = prim::lds_object<ScopeGroup>();
  const uint32_t tid = scope_tid();
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  const uint64_t c0 = (uint64_t)c * kScopeChunk;
  load_stored_kinds(a, n, g, tid, c);
  DepthFn f = fn_id();
  for (int k = 0; k < kScopePer; k++) f = fn_then(f, fn_of_entry(g.K[tid * kScopePer + k]));
  const DepthFn ex = group_exclusive(g, tid, f);
  int64_t d = fn_apply(ex, unpack64(prim::ld_pair(a.in_depth + c)));
  // the level offset of the run's first entry's document (batches)
  uint32_t off = 0;
  const uint64_t r0 = c0 + (uint64_t)tid * kScopePer;
  if (BATCH && r0 < n) off = prim::load4(reinterpret_cast<const uint8_t*>(a.vstart + prim::load4(reinterpret_cast<const uint8_t*>(a.docid + r0))));
  uint32_t lo_level = kNoLevel;
  for (int k = 0; k < kScopePer; k++) {
    const uint32_t j = tid * kScopePer + (uint32_t)k;
    const uint32_t kb = g.K[j];
    uint32_t kd = kb & kTokMask, level = kNoLevel;
    if (kb & kDocStartBit) {
      d = 0;
      off = (uint32_t)(c0 + j);
    }
    const uint32_t root = d == 0 ? kRootBit : 0u;
    if (kd == kOpenSq || kd == kOpenCu) {
      level = off + (uint32_t)d;
      d++;
    } else if (kd == kCloseSq || kd == kCloseCu) {
      if (d > 0) {
        d--;
        level = off + (uint32_t)d;
      } else {
        kd = kOther;  // a closer with nothing open: left unlinked
        if (c0 + j < n) prim::or_agent32(err_of<BATCH>(a, c0 + j), kErrUnbalanced);
      }
    }
    g.L[j] = level;
    g.K[j] = (uint8_t)(kd | root | (kb & (kDocStartBit | kDocEndBit)));
    if (level < lo_level) lo_level = level;
  }
  g.m[tid] = lo_level;
  prim::sync();
  // the chunk's levels, kinds and cleared links go out as consecutive words,
  // four entries per thread and store (bytes past n are left as they were)
  const uint32_t* kw = reinterpret_cast<const uint32_t*>(g.K);
  for (uint32_t q = tid; q < (uint32_t)kScopeChunk / 4; q += kScopeThreads) {
    const uint64_t e = c0 + 4 * (uint64_t)q;
    if (e >= n) break;
    if (e + 4 <= n) {
      prim::st_out4(a.lev + e, uint4{g.L[4 * q], g.L[4 * q + 1], g.L[4 * q + 2], g.L[4 * q + 3]});
      prim::st_out(reinterpret_cast<uint32_t*>(a.kind + e), kw[q]);
      prim::st_out4(a.match + e, uint4{kUnlinked, kUnlinked, kUnlinked, kUnlinked});
      continue;
    }
    for (uint32_t k = 0; k < 4u && e + k < n; k++) {
      prim::st_out(a.lev + e + k, g.L[4 * q + k]);
      prim::st_byte(a.kind + e + k, g.K[4 * q + k]);
      prim::st_out(a.match + e + k, kUnlinked);
    }
  }
  for (uint32_t s = kScopeThreads / 2; s > 0; s >>= 1) {
    if (tid < s && g.m[tid + s] < g.m[tid]) g.m[tid] = g.m[tid + s];
    prim::sync();
  }
  if (tid == 0) prim::st_out(a.chunk_min + c, g.m[0]);
  prim::sync();
  }
}

// Links opener i (token ki) with closer k.  The closer's kind byte also
// learns whether the opener follows a colon (in its own document); only this
// call writes it (the kernel owning k's chunk has staged its kinds before
// linking).
template <bool BATCH>
JSIDX_DEV void link(const ScopeArgs& a, uint32_t i, uint32_t k, uint32_t ki) {
  prim::st_out(a.match + i, k);
  prim::st_out(a.match + k, i);
  const uint32_t kb = prim::load1(a.kind + k);
  const uint32_t kk = kb & kTokMask;
  if ((ki == kOpenCu) != (kk == kCloseCu)) prim::or_agent32(err_of<BATCH>(a, i), kErrMismatched);
  const bool first = BATCH && (prim::load1(a.kind + i) & kDocStartBit) != 0u;
  if (i > 0 && !first && (prim::load1(a.kind + i - 1) & kTokMask) == kColon) prim::st_byte(a.kind + k, kb | kMemberBit);
}

// 4. Each opener's closer inside its own chunk, searched in LDS; openers whose
//    scope leaves the chunk are queued (one workgroup per chunk).
template <bool BATCH>
JSIDX_DEVFN void scope_local(const ScopeArgs& a) {
  ScopeGroup& g = prim::lds_object<ScopeGroup>();
  const uint32_t tid = scope_tid();
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  const uint64_t c0 = (uint64_t)c * kScopeChunk;
  const uint32_t cend = n - c0 < (uint64_t)kScopeChunk ? (uint32_t)(n - c0) : (uint32_t)kScopeChunk;
  // levels and whole kind bytes, four entries per load (past the end: no
  // level, kOther)
  {
    constexpr int kR = kScopeChunk / 4 / kScopeThreads;
    uint4 lq[kR];
    uint32_t kq[kR];
#pragma unroll
    for (int r = 0; r < kR; r++) {
      const uint32_t j = 4u * (tid + (uint32_t)r * kScopeThreads);
      if (j + 4 <= cend) {
        lq[r] = prim::load16(reinterpret_cast<const uint8_t*>(a.lev + c0 + j));
        kq[r] = prim::load4(a.kind + c0 + j);
      } else {
        uint32_t l[4], kw = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const bool in = j + k < cend;
          l[k] = in ? prim::load4(reinterpret_cast<const uint8_t*>(a.lev + c0 + j + k)) : kNoLevel;
          kw |= (in ? prim::load1(a.kind + c0 + j + k) : (uint32_t)kOther) << (8 * k);
        }
        lq[r] = uint4{l[0], l[1], l[2], l[3]};
        kq[r] = kw;
      }
    }
    uint32_t* kw = reinterpret_cast<uint32_t*>(g.K);
#pragma unroll
    for (int r = 0; r < kR; r++) {
      const uint32_t q = tid + (uint32_t)r * kScopeThreads;
      g.L[4 * q] = lq[r].x;
      g.L[4 * q + 1] = lq[r].y;
      g.L[4 * q + 2] = lq[r].z;
      g.L[4 * q + 3] = lq[r].w;
      kw[q] = kq[r];
    }
  }
  prim::sync();
  // lowest level of each thread's run of kScopePer entries
  uint32_t gmin = kNoLevel;
  for (int k = 0; k < kScopePer; k++) {
    const uint32_t v = g.L[tid * kScopePer + k];
    gmin = v < gmin ? v : gmin;
  }
  g.m[tid] = gmin;
  prim::sync();
  if (tid < (uint32_t)(kScopeThreads / kScopeRunGroup)) {
    uint32_t m2 = kNoLevel;
    for (int k = 0; k < kScopeRunGroup; k++) {
      const uint32_t v = g.m[tid * kScopeRunGroup + k];
      m2 = v < m2 ? v : m2;
    }
    g.m2[tid] = m2;
  }
  prim::sync();
  for (int k = 0; k < kScopePer; k++) {
    const uint32_t j = tid * kScopePer + (uint32_t)k;
    if (j >= cend) break;
    const uint32_t i = (uint32_t)(c0 + j);
    const uint32_t ki = g.K[j] & kTokMask;
    if (ki != kOpenSq && ki != kOpenCu) continue;
    const uint32_t lv = g.L[j];
    // the rest of this run, then the rest of its group of runs by their
    // lowest levels, then whole groups, then the runs of the first group
    // that can hold the closer, then inside the first run that can
    uint32_t p = j + 1;
    const uint32_t run_end = (tid + 1) * kScopePer;
    while (p < run_end && g.L[p] > lv) p++;
    if (p >= run_end) {
      uint32_t r = tid + 1;
      const uint32_t gend = (tid / kScopeRunGroup + 1) * kScopeRunGroup;
      while (r < gend && g.m[r] > lv) r++;
      if (r == gend) {
        uint32_t gi = gend / kScopeRunGroup;
        while (gi < (uint32_t)(kScopeThreads / kScopeRunGroup) && g.m2[gi] > lv) gi++;
        r = gi * kScopeRunGroup;
        if (r < (uint32_t)kScopeThreads)
          while (g.m[r] > lv) r++;  // inside group gi: its lowest level is at most lv
      }
      p = r * kScopePer;
      if (r < (uint32_t)kScopeThreads)
        while (g.L[p] > lv) p++;  // ends inside run r: its lowest level is at most lv
    }
    if (p < cend) {
      // as link(), with the kind bytes from LDS (only this call changes the
      // closer's)
      const uint32_t k = (uint32_t)(c0 + p), kb = g.K[p];
      prim::st_out(a.match + i, k);
      prim::st_out(a.match + k, i);
      if ((ki == kOpenCu) != ((kb & kTokMask) == kCloseCu)) prim::or_agent32(err_of<BATCH>(a, i), kErrMismatched);
      const bool first = BATCH && (g.K[j] & kDocStartBit) != 0u;
      const uint32_t prev = j ? g.K[j - 1] : i ? prim::load1(a.kind + i - 1) : (uint32_t)kOther;
      if (i > 0 && !first && (prev & kTokMask) == kColon) prim::st_byte(a.kind + k, kb | kMemberBit);
    } else {
      const uint32_t q = prim::add_agent32(a.qcount, 1u);
      prim::st_out(a.queue + q, i);
    }
  }
  prim::sync();
  }
}

// 5. Queued openers: the first later chunk whose lowest level is at most the
//    opener's, then the first such entry in it; one wave per opener, 64
//    chunks or entries per step.  (In a batch the search stops at the chunk
//    of the document's last entry.)
template <bool BATCH>
JSIDX_DEVFN void scope_far(const ScopeArgs& a) {
  const uint32_t lane = prim::lane();
  const uint32_t qn = prim::readlane(prim::ld_agent32(a.qcount), 0);
  const uint32_t n = prim::readlane(n_of<BATCH>(a), 0);
  const uint32_t waves_per_group = kScopeThreads / kScopeWave;
  const uint32_t nw = prim::grid() * waves_per_group;
  for (uint32_t q = prim::block() * waves_per_group + prim::wave_id(); q < qn; q += nw) {
    const uint32_t i = prim::readlane(prim::load4(reinterpret_cast<const uint8_t*>(a.queue + q)), 0);
    const uint32_t lv = prim::readlane(prim::load4(reinterpret_cast<const uint8_t*>(a.lev + i)), 0);
    const uint32_t ki = prim::readlane(prim::load1(a.kind + i) & kTokMask, 0);
    uint64_t end = n;  // entries [i, end) can hold the closer
    if (BATCH) {
      const uint32_t d = prim::readlane(prim::load4(reinterpret_cast<const uint8_t*>(a.docid + i)), 0);
      end = prim::readlane(prim::load4(reinterpret_cast<const uint8_t*>(a.vstart + d + 1)), 0);
    }
    const uint64_t cend = (end + kScopeChunk - 1) / kScopeChunk;
    int64_t c2 = -1;
    for (uint64_t base = (uint64_t)i / kScopeChunk + 1; base < cend; base += kScopeWave) {
      const uint64_t cc = base + lane;
      const bool ok = cc < cend && prim::load4(reinterpret_cast<const uint8_t*>(a.chunk_min + cc)) <= lv;
      const uint64_t bm = prim::ballot(ok);
      if (bm) {
        c2 = (int64_t)(base + (uint64_t)__builtin_ctzll(bm));
        break;
      }
    }
    int64_t found = -1;
    if (c2 >= 0) {
      const uint64_t start = (uint64_t)c2 * kScopeChunk;
      const uint64_t stop = start + kScopeChunk < end ? start + kScopeChunk : end;
      for (uint64_t p0 = start; p0 < stop; p0 += kScopeWave) {
        const uint64_t p = p0 + lane;
        const bool ok = p < stop && prim::load4(reinterpret_cast<const uint8_t*>(a.lev + p)) <= lv;
        const uint64_t bm = prim::ballot(ok);
        if (bm) {
          found = (int64_t)(p0 + (uint64_t)__builtin_ctzll(bm));
          break;
        }
      }
    }
    if (lane == 0) {
      if (found >= 0) link<BATCH>(a, i, (uint32_t)found, ki);
      else prim::or_agent32(err_of<BATCH>(a, i), kErrUnbalanced);
    }
  }
}

// ---- Structure ---------------------------------------------------------
// The entries' tokens must form one JSON value (the grammar of values,
// objects and arrays recalled in Sec. 1, which the paper's stage 2 enforces
// while it builds the tape, Sec. 3.2).  Each entry is judged with the few
// entries around it; the scope of a comma needs no search: the element before
// the comma ends just before it, and it is an object member exactly when its
// value (an atom or string there, or the scope ending at a closer there)
// follows a colon, which link() recorded on the closer.  Every comma must be
// followed by an element of the same form; the first element after '{' must
// be a member and after '[' a plain value, so by induction every element has
// the form of its scope.  A member is a string followed by a colon.

// Entry i of chunk c0 (i in [c0 - 4, c0 + kScopeChunk + 3]) from the staged
// kinds: its token, kRootBit, or 0xFF outside the index.
struct Staged {
  const uint8_t* K;
  int64_t c0;
  JSIDX_DEV uint32_t raw(int64_t i) const { return K[i - c0 + 4]; }
  JSIDX_DEV uint32_t tok(int64_t i) const { const uint32_t k = raw(i); return k == 0xFFu ? k : k & kTokMask; }
};

// The check as a table: each entry gets a class as the entry being checked
// (its token, with strings split into keys -- followed by a colon -- and
// values, and commas at depth 0 apart) and a class as the predecessor of the
// next entry (its token, with strings split the same way and commas split by
// the form of the element before them: after an object member, after a plain
// value).  An entry is valid iff its class is allowed after its
// predecessor's.
enum : uint32_t {  // as the entry checked (tokens 0..6 keep their values)
  cStrVal = 7, cStrKey = 8, cRootComma = 9
};
enum : uint32_t {  // as the predecessor (tokens 0..5 keep their values)
  pCommaArr = 6, pStrVal = 7, pStrKey = 8, pCommaObj = 9, pStart = 10
};
constexpr uint32_t cls_bit(uint32_t c) { return 1u << c; }
constexpr uint32_t kValueStarts = cls_bit(kOther) | cls_bit(kOpenSq) | cls_bit(kOpenCu) | cls_bit(cStrVal);
constexpr uint32_t kAfterValue = cls_bit(kComma) | cls_bit(kCloseSq) | cls_bit(kCloseCu);
// allowed classes after each predecessor class, 10 bits each
constexpr uint64_t kAllowLo =  // predecessors 0..5: atom [ { ] } :
    ((uint64_t)kAfterValue << 0) | ((uint64_t)(kValueStarts | cls_bit(kCloseSq)) << 10) |
    ((uint64_t)(cls_bit(cStrKey) | cls_bit(kCloseCu)) << 20) | ((uint64_t)kAfterValue << 30) |
    ((uint64_t)kAfterValue << 40) | ((uint64_t)kValueStarts << 50);
constexpr uint64_t kAllowHi =  // predecessors 6..10: array comma, value, key, object comma, start
    ((uint64_t)kValueStarts << 0) | ((uint64_t)kAfterValue << 10) | ((uint64_t)cls_bit(kColon) << 20) |
    ((uint64_t)cls_bit(cStrKey) << 30) | ((uint64_t)kValueStarts << 40);
constexpr uint32_t kLastAllowed = cls_bit(kOther) | cls_bit(cStrVal) | cls_bit(kCloseSq) | cls_bit(kCloseCu);

JSIDX_DEV bool allowed(uint32_t pc, uint32_t cc) {
  const uint64_t row = pc < 6 ? kAllowLo >> (10 * pc) : kAllowHi >> (10 * (pc - 6));
  return ((row >> cc) & 1u) != 0u;
}

// Structure check of entry i (entries i - 3 .. i + 1 staged; n entries).  In
// a batch, entries of other documents count as outside the index.
template <bool BATCH>
JSIDX_DEV bool entry_ok(uint32_t n, const Staged& st, int64_t i) {
  const uint32_t r0 = st.raw(i);
  const bool first = BATCH ? (r0 & kDocStartBit) != 0u : i == 0;
  const bool last = BATCH ? (r0 & kDocEndBit) != 0u : (uint64_t)i + 1 == n;
  // i - 2 and i - 3 are in i's document only if no document starts after them
  const bool in2 = !BATCH || !first ? !BATCH || (st.raw(i - 1) & kDocStartBit) == 0u : false;
  const bool in3 = in2 && (!BATCH || (st.raw(i - 2) & kDocStartBit) == 0u);
  const uint32_t t = st.tok(i), nxt = last ? 0xFFu : st.tok(i + 1);
  uint32_t cc = t;
  if (t == kStr) cc = nxt == kColon ? cStrKey : cStrVal;
  else if (t == kComma && (r0 & kRootBit)) cc = cRootComma;
  uint32_t pc = pStart;
  if (!first) {
    const uint32_t p = st.tok(i - 1);
    pc = p;
    if (p == kStr) {
      pc = t == kColon ? pStrKey : pStrVal;
    } else if (p == kComma) {
      // the element before the comma ends at i - 2: an object member iff its
      // value (an atom or string there, or the scope a closer there ends)
      // follows a colon
      const uint32_t te = in2 ? st.tok(i - 2) : 0xFFu;
      const bool member = (te == kCloseSq || te == kCloseCu) ? (st.raw(i - 2) & kMemberBit) != 0u
                                                              : (in3 ? st.tok(i - 3) : 0xFFu) == kColon;
      pc = member ? pCommaObj : pCommaArr;
    }
  }
  bool ok = allowed(pc, cc);
  if (last) ok = ok && (kLastAllowed >> cc) & 1u;
  return ok;
}

// 6. The structure check, after the links (one workgroup per chunk, kinds
//    staged in LDS with coalesced word loads; the rule of entry i reads
//    entries i - 3 to i + 1 only).  Unbalanced or mismatched brackets are a
//    syntax error too (for a batch, scope_batch_finish adds that).
template <bool BATCH>
JSIDX_DEVFN void scope_check(const ScopeArgs& a) {
  ScopeCheckLds& g = prim::lds_object<ScopeCheckLds>();
  const uint32_t tid = scope_tid();
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  const int64_t c0 = (int64_t)c * kScopeChunk;
  if (!BATCH && c == 0 && tid == 0 && (prim::ld_agent32(a.err) & (kErrUnbalanced | kErrMismatched)))
    prim::or_agent32(a.err, kErrSyntax);
  // words of the kind array; bytes outside [0, n) read as 0xFF (the array's
  // allocation is padded to 256 bytes, so a word holding byte n - 1 is inside)
  for (uint32_t w = tid; w < (uint32_t)kCheckWords; w += kScopeThreads) {
    const int64_t b = c0 - 4 + 4 * (int64_t)w;
    uint32_t v = 0xFFFFFFFFu;
    if (b >= 0 && (uint64_t)b < n) {
      v = prim::load4(a.kind + b);
      const uint64_t valid = n - (uint64_t)b;
      if (valid < 4) v |= 0xFFFFFFFFu << (8 * valid);
    }
    g.W[w] = v;
  }
  prim::sync();
  const Staged st{reinterpret_cast<const uint8_t*>(g.W), c0};
  bool ok = true;
  for (uint32_t j = tid; j < (uint32_t)kScopeChunk; j += kScopeThreads) {
    const int64_t i = c0 + (int64_t)j;
    if ((uint64_t)i >= n) break;
    const bool e = entry_ok<BATCH>(n, st, i);
    if (BATCH && !e) prim::or_agent32(err_of<true>(a, (uint64_t)i), kErrSyntax);
    ok = e && ok;
  }
  if (!BATCH && prim::ballot(!ok) != 0ull && prim::lane() == 0) prim::or_agent32(a.err, kErrSyntax);
  prim::sync();
  }
}

// ---- Batches ---------------------------------------------------------------
// 0. The first virtual entry of each document: the entry counts summed per
//    2048 documents (scope_batch_sums), the sums scanned with the totals and
//    the queue emptied (scope_batch_bases, one workgroup), then every
//    document's start and cleared flags (scope_batch_starts; an empty index
//    is a syntax error).  A batch with more entries than the workspace holds
//    is not linked: every document gets JSIDX_ERR_CAPACITY (0x80000000) and
//    the kernels after these do nothing.
constexpr uint32_t kErrCapacity = 0x80000000u;
JSIDX_DEVFN void scope_batch_sums(const ScopeArgs& a) { docscan_sums(a.dn, a.ndocs, false, a.part); }

JSIDX_DEVFN void scope_batch_bases(const ScopeArgs& a) {
  const uint64_t total = docscan_bases((uint32_t)docscan_groups(a.ndocs), a.part);
  if (scope_tid() == 0) {
    const bool over = total > (uint64_t)a.cap;
    if (!over) prim::st_out(a.vstart + a.ndocs, (uint32_t)total);
    prim::st_out(a.vn, over ? 0u : (uint32_t)total);
    prim::st_out(a.vn + 1, over ? 0u : (uint32_t)((total + kScopeChunk - 1) / kScopeChunk));
    prim::st_out(a.vn + 2, over ? 1u : 0u);
    prim::st_out(a.qcount, 0u);
  }
}

JSIDX_DEVFN void scope_batch_starts(const ScopeArgs& a) {
  const bool over = prim::ld_agent32(a.vn + 2) != 0u;
  docscan_starts(a.dn, a.ndocs, false, a.part, [&](uint64_t d, uint64_t start, uint32_t cnt) {
    if (!over) prim::st_out(a.vstart + d, (uint32_t)start);
    prim::st_out(a.err + d, over ? kErrCapacity : (cnt ? 0u : kErrSyntax));
  });
}

// 1b. Each document's entries into the virtual sequence: kind bytes (with
//     the first and last entry of the document marked) and document numbers,
//     one wave per document.
JSIDX_DEVFN void scope_batch_compact(const ScopeArgs& a) {
  const uint32_t lane = prim::lane();
  if (prim::ld_agent32(a.vn + 1) == 0u) return;
  const uint32_t waves_per_group = kScopeThreads / kScopeWave;
  const uint32_t nw = prim::grid() * waves_per_group;
  for (uint32_t d = prim::block() * waves_per_group + prim::wave_id(); d < a.ndocs; d += nw) {
    const uint64_t base = prim::load8(a.offsets + d), len = prim::load8(a.offsets + d + 1) - base;
    const uint32_t nd = prim::load4(reinterpret_cast<const uint8_t*>(a.dn + d));
    const uint32_t v0 = prim::load4(reinterpret_cast<const uint8_t*>(a.vstart + d));
    // four steps of 64 entries at a time: their positions, then their bytes,
    // each set of loads in flight together
    constexpr uint32_t kU = 4;
    for (uint32_t j0 = 0; j0 < nd; j0 += kU * kScopeWave) {
      uint32_t pj[kU], bj[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) {
        const uint32_t j = j0 + u * kScopeWave + lane;
        pj[u] = j < nd ? prim::load4(reinterpret_cast<const uint8_t*>(a.idx + base + j)) : 0xFFFFFFFFu;
      }
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) bj[u] = (uint64_t)pj[u] < len ? prim::load1(a.buf + base + pj[u]) : 0x100u;
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) {
        const uint32_t j = j0 + u * kScopeWave + lane;
        if (j >= nd) continue;
        const uint32_t b = bj[u];
        uint32_t k = b == 0x5Bu ? kOpenSq : b == 0x7Bu ? kOpenCu : b == 0x5Du ? kCloseSq : b == 0x7Du ? kCloseCu
                   : b == 0x3Au ? kColon : b == 0x2Cu ? kComma : b == 0x22u ? kStr : kOther;
        if (j == 0) k |= kDocStartBit;
        if (j + 1 == nd) k |= kDocEndBit;
        prim::st_byte(a.kind + v0 + j, k);
        prim::st_out(a.docid + v0 + j, d);
      }
    }
  }
}

// 7. Links back into the batch layout (document-relative entry numbers at
//    out_match + offsets[d]) and the flags completed: unbalanced or
//    mismatched brackets are a syntax error.  One wave per document.
JSIDX_DEVFN void scope_batch_finish(const ScopeArgs& a) {
  const uint32_t lane = prim::lane();
  if (prim::ld_agent32(a.vn + 1) == 0u) return;
  const uint32_t waves_per_group = kScopeThreads / kScopeWave;
  const uint32_t nw = prim::grid() * waves_per_group;
  for (uint32_t d = prim::block() * waves_per_group + prim::wave_id(); d < a.ndocs; d += nw) {
    const uint64_t base = prim::load8(a.offsets + d);
    const uint32_t nd = prim::load4(reinterpret_cast<const uint8_t*>(a.dn + d));
    const uint32_t v0 = prim::load4(reinterpret_cast<const uint8_t*>(a.vstart + d));
    constexpr uint32_t kU = 4;  // four steps of 64 entries, their loads in flight together
    for (uint32_t j0 = 0; j0 < nd; j0 += kU * kScopeWave) {
      uint32_t mj[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) {
        const uint32_t j = j0 + u * kScopeWave + lane;
        mj[u] = j < nd ? prim::load4(reinterpret_cast<const uint8_t*>(a.match + v0 + j)) : kUnlinked;
      }
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) {
        const uint32_t j = j0 + u * kScopeWave + lane;
        if (j < nd) prim::st_out(a.out_match + base + j, mj[u] == kUnlinked ? kUnlinked : mj[u] - v0);
      }
    }
    if (lane == 0) {
      const uint32_t e = prim::ld_agent32(a.err + d);
      if (e & (kErrUnbalanced | kErrMismatched)) prim::st_out(a.err + d, e | kErrSyntax);
    }
  }
}

}  // namespace jsidx
