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
#pragma once

#include "jsidx_device.h"

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
// Token of an index entry: atoms (numbers, literals, anything else) are kOther.
enum : uint32_t { kOther = 0, kOpenSq = 1, kOpenCu = 2, kCloseSq = 3, kCloseCu = 4, kColon = 5, kComma = 6, kStr = 7 };

struct DepthFn {  // x -> max(x + a, b)
  int64_t a, b;
};
constexpr int64_t kNegInf = -(1ll << 62);

JSIDX_DEV DepthFn fn_id() { return DepthFn{0, kNegInf}; }
JSIDX_DEV DepthFn fn_then(const DepthFn& f, const DepthFn& g) {  // f, then g
  const int64_t fb = f.b + g.a;
  return DepthFn{f.a + g.a, fb > g.b ? fb : g.b};
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
  uint32_t* qt;         // per entry: threshold of its search (openers, commas)
  uint32_t* dep;        // per entry: depth before it
  uint8_t* kind;        // per entry: token
  uint8_t* ck;          // per comma: the closing bracket of its scope
  uint32_t* queue;      // per entry at most
};

// Workspace layout for n entries (byte offsets; host side).
struct ScopeLayout {
  uint64_t chunk_fn, in_depth, chunk_min, qcount, lev, qt, dep, queue, kind, ck, total;
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
  L.qt = o; o = scope_align256(o + n * 4);
  L.dep = o; o = scope_align256(o + n * 4);
  L.queue = o; o = scope_align256(o + n * 4);
  L.kind = o; o = scope_align256(o + n);
  L.ck = o; o = scope_align256(o + n);
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

JSIDX_DEV uint32_t kind_at(const ScopeArgs& a, uint32_t i) {
  const uint32_t p = prim::load4(reinterpret_cast<const uint8_t*>(a.idx + i));
  if ((uint64_t)p >= a.len) return kOther;  // not a position of this document
  const uint32_t b = prim::load1(a.buf + p);
  return b == 0x5Bu ? kOpenSq : b == 0x7Bu ? kOpenCu : b == 0x5Du ? kCloseSq : b == 0x7Du ? kCloseCu
       : b == 0x3Au ? kColon : b == 0x2Cu ? kComma : b == 0x22u ? kStr : kOther;
}

struct ScopeGroup {
  DepthFn f[kScopeThreads];
  uint32_t m[kScopeThreads];
  uint32_t L[kScopeChunk];  // levels of the chunk's entries
  uint32_t T[kScopeChunk];  // search thresholds (scope_local), depths (scope_levels)
  uint8_t K[kScopeChunk];   // tokens of the chunk's entries
};

JSIDX_DEV uint32_t scope_tid() { return prim::wave_id() * kScopeWave + prim::lane(); }

// The kinds of chunk c's entries into LDS: consecutive threads read
// consecutive entries (coalesced), then each thread works on its own run of
// kScopePer entries in LDS.
JSIDX_DEV void load_kinds(const ScopeArgs& a, ScopeGroup& g, uint32_t tid, uint32_t c) {
  const uint64_t c0 = (uint64_t)c * kScopeChunk;
  for (uint32_t j = tid; j < (uint32_t)kScopeChunk; j += kScopeThreads)
    g.K[j] = (uint8_t)(c0 + j < a.n ? kind_at(a, (uint32_t)(c0 + j)) : kOther);
  prim::sync();
}

// Ordered inclusive scan of the workgroup's per-thread functions; returns the
// composition of the threads before this one.
JSIDX_DEV DepthFn group_exclusive(ScopeGroup& g, uint32_t tid, DepthFn mine) {
  g.f[tid] = mine;
  prim::sync();
  for (uint32_t s = 1; s < (uint32_t)kScopeThreads; s <<= 1) {
    const DepthFn t = tid >= s ? fn_then(g.f[tid - s], g.f[tid]) : g.f[tid];
    prim::sync();
    g.f[tid] = t;
    prim::sync();
  }
  const DepthFn ex = tid ? g.f[tid - 1] : fn_id();
  prim::sync();
  return ex;
}

// 1. The composed depth function of each chunk (one workgroup per chunk).
JSIDX_DEVFN void scope_chunk_fn(const ScopeArgs& a) {
  ScopeGroup& g = prim::lds_object<ScopeGroup>();
  const uint32_t tid = scope_tid(), c = prim::block();
  load_kinds(a, g, tid, c);
  DepthFn f = fn_id();
  for (int k = 0; k < kScopePer; k++) f = fn_then(f, fn_of(g.K[tid * kScopePer + k]));
  const DepthFn ex = group_exclusive(g, tid, f);
  if (tid == kScopeThreads - 1) {
    const DepthFn all = fn_then(ex, f);
    prim::st_pair(a.chunk_fn + 2 * (uint64_t)c, pack64(all.a).x, pack64(all.a).y);
    prim::st_pair(a.chunk_fn + 2 * (uint64_t)c + 1, pack64(all.b).x, pack64(all.b).y);
  }
}

// 2. The depth entering each chunk (one workgroup); also clears the flags and
//    the queue for the kernels after it.
JSIDX_DEVFN void scope_scan(const ScopeArgs& a) {
  ScopeGroup& g = prim::lds_object<ScopeGroup>();
  const uint32_t tid = scope_tid();
  const uint32_t per = (a.nchunks + kScopeThreads - 1) / kScopeThreads;
  const uint64_t lo = (uint64_t)tid * per;
  const uint64_t hi = lo + per < a.nchunks ? lo + per : a.nchunks;
  DepthFn f = fn_id();
  for (uint64_t c = lo; c < hi; c++) {
    const DepthFn fc{unpack64(prim::ld_pair(a.chunk_fn + 2 * c)), unpack64(prim::ld_pair(a.chunk_fn + 2 * c + 1))};
    f = fn_then(f, fc);
  }
  const DepthFn ex = group_exclusive(g, tid, f);
  int64_t x = fn_apply(ex, 0);
  for (uint64_t c = lo; c < hi; c++) {
    prim::st_pair(a.in_depth + c, pack64(x).x, pack64(x).y);
    const DepthFn fc{unpack64(prim::ld_pair(a.chunk_fn + 2 * c)), unpack64(prim::ld_pair(a.chunk_fn + 2 * c + 1))};
    x = fn_apply(fc, x);
  }
  if (tid == 0) {
    prim::st_out(a.err, a.n ? 0u : kErrSyntax);  // an empty index holds no value
    prim::st_out(a.qcount, 0u);
  }
}

// 3. Levels and kinds of the entries, the lowest level of each chunk, and
//    every link cleared (one workgroup per chunk).
JSIDX_DEVFN void scope_levels(const ScopeArgs& a) {
  ScopeGroup& g = prim::lds_object<ScopeGroup>();
  const uint32_t tid = scope_tid(), c = prim::block();
  const uint64_t c0 = (uint64_t)c * kScopeChunk;
  load_kinds(a, g, tid, c);
  DepthFn f = fn_id();
  for (int k = 0; k < kScopePer; k++) f = fn_then(f, fn_of(g.K[tid * kScopePer + k]));
  const DepthFn ex = group_exclusive(g, tid, f);
  int64_t d = fn_apply(ex, unpack64(prim::ld_pair(a.in_depth + c)));
  uint32_t lo_level = kNoLevel, unmatched = 0;
  for (int k = 0; k < kScopePer; k++) {
    const uint32_t j = tid * kScopePer + (uint32_t)k;
    uint32_t kd = g.K[j], level = kNoLevel;
    g.T[j] = (uint32_t)d;
    if (kd == kOpenSq || kd == kOpenCu) {
      level = (uint32_t)d;
      d++;
    } else if (kd == kCloseSq || kd == kCloseCu) {
      if (d > 0) {
        d--;
        level = (uint32_t)d;
      } else {
        kd = kOther;  // a closer with nothing open: left unlinked
        unmatched = 1;
      }
    }
    g.L[j] = level;
    g.K[j] = (uint8_t)kd;
    if (level < lo_level) lo_level = level;
  }
  if (unmatched) prim::or_agent32(a.err, kErrUnbalanced);
  g.m[tid] = lo_level;
  prim::sync();
  // the chunk's levels, kinds and cleared links go out as consecutive words
  for (uint32_t j = tid; j < (uint32_t)kScopeChunk; j += kScopeThreads) {
    if (c0 + j >= a.n) break;
    const uint32_t kd = g.K[j], dj = g.T[j];
    // search threshold: an opener looks for its closer, a comma for the
    // closer of its scope (none at the root)
    const uint32_t qt = (kd == kOpenSq || kd == kOpenCu) ? dj : (kd == kComma && dj > 0 ? dj - 1u : kNoLevel);
    prim::st_out(a.lev + c0 + j, g.L[j]);
    prim::st_out(a.qt + c0 + j, qt);
    prim::st_out(a.dep + c0 + j, dj);
    prim::st_byte(a.kind + c0 + j, kd);
    prim::st_byte(a.ck + c0 + j, 0u);
    prim::st_out(a.match + c0 + j, kUnlinked);
  }
  for (uint32_t s = kScopeThreads / 2; s > 0; s >>= 1) {
    if (tid < s && g.m[tid + s] < g.m[tid]) g.m[tid] = g.m[tid + s];
    prim::sync();
  }
  if (tid == 0) prim::st_out(a.chunk_min + c, g.m[0]);
}

// The search of entry i (token ki) ended at entry k: an opener is linked with
// its closer, a comma learns the closer of its scope.
JSIDX_DEV void resolve(const ScopeArgs& a, uint32_t i, uint32_t k, uint32_t ki) {
  const uint32_t kk = prim::load1(a.kind + k);
  if (ki == kComma) {
    prim::st_byte(a.ck + i, kk);
    return;
  }
  prim::st_out(a.match + i, k);
  prim::st_out(a.match + k, i);
  if ((ki == kOpenCu) != (kk == kCloseCu)) prim::or_agent32(a.err, kErrMismatched);
}

// 4. Each opener's closer inside its own chunk, searched in LDS; openers whose
//    scope leaves the chunk are queued (one workgroup per chunk).
JSIDX_DEVFN void scope_local(const ScopeArgs& a) {
  ScopeGroup& g = prim::lds_object<ScopeGroup>();
  const uint32_t tid = scope_tid(), c = prim::block();
  const uint64_t c0 = (uint64_t)c * kScopeChunk;
  const uint32_t cend = a.n - c0 < (uint64_t)kScopeChunk ? (uint32_t)(a.n - c0) : (uint32_t)kScopeChunk;
  for (uint32_t j = tid; j < (uint32_t)kScopeChunk; j += kScopeThreads) {
    g.L[j] = j < cend ? prim::load4(reinterpret_cast<const uint8_t*>(a.lev + c0 + j)) : kNoLevel;
    g.T[j] = j < cend ? prim::load4(reinterpret_cast<const uint8_t*>(a.qt + c0 + j)) : kNoLevel;
    g.K[j] = (uint8_t)(j < cend ? prim::load1(a.kind + c0 + j) : kOther);
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
  for (int k = 0; k < kScopePer; k++) {
    const uint32_t j = tid * kScopePer + (uint32_t)k;
    if (j >= cend) break;
    const uint32_t i = (uint32_t)(c0 + j);
    const uint32_t ki = g.K[j];
    const uint32_t lv = g.T[j];
    if (lv == kNoLevel) continue;  // neither an opener nor a comma inside a scope
    // the rest of this run, then whole runs by their lowest level, then
    // inside the first run that can hold the closer
    uint32_t p = j + 1;
    const uint32_t run_end = (tid + 1) * kScopePer;
    while (p < run_end && g.L[p] > lv) p++;
    if (p >= run_end) {
      uint32_t r = tid + 1;
      while (r < (uint32_t)kScopeThreads && g.m[r] > lv) r++;
      p = r * kScopePer;
      if (r < (uint32_t)kScopeThreads)
        while (g.L[p] > lv) p++;  // ends inside run r: its lowest level is at most lv
    }
    if (p < cend) {
      resolve(a, i, (uint32_t)(c0 + p), ki);
    } else {
      const uint32_t q = prim::add_agent32(a.qcount, 1u);
      prim::st_out(a.queue + q, i);
    }
  }
}

// 5. Queued openers: the first later chunk whose lowest level is at most the
//    opener's, then the first such entry in it; one wave per opener, 64
//    chunks or entries per step.
JSIDX_DEVFN void scope_far(const ScopeArgs& a) {
  const uint32_t lane = prim::lane();
  const uint32_t qn = prim::readlane(prim::ld_agent32(a.qcount), 0);
  const uint32_t waves_per_group = kScopeThreads / kScopeWave;
  const uint32_t nw = prim::grid() * waves_per_group;
  for (uint32_t q = prim::block() * waves_per_group + prim::wave_id(); q < qn; q += nw) {
    const uint32_t i = prim::readlane(prim::load4(reinterpret_cast<const uint8_t*>(a.queue + q)), 0);
    const uint32_t lv = prim::readlane(prim::load4(reinterpret_cast<const uint8_t*>(a.qt + i)), 0);
    const uint32_t ki = prim::readlane(prim::load1(a.kind + i), 0);
    int64_t c2 = -1;
    for (uint64_t base = (uint64_t)i / kScopeChunk + 1; base < a.nchunks; base += kScopeWave) {
      const uint64_t cc = base + lane;
      const bool ok = cc < a.nchunks && prim::load4(reinterpret_cast<const uint8_t*>(a.chunk_min + cc)) <= lv;
      const uint64_t bm = prim::ballot(ok);
      if (bm) {
        c2 = (int64_t)(base + (uint64_t)__builtin_ctzll(bm));
        break;
      }
    }
    if (c2 < 0) {  // an opener never closed, or a comma whose scope never closes
      if (lane == 0) prim::or_agent32(a.err, kErrUnbalanced);
      continue;
    }
    const uint64_t start = (uint64_t)c2 * kScopeChunk;
    const uint64_t stop = start + kScopeChunk < a.n ? start + kScopeChunk : a.n;
    int64_t found = -1;
    for (uint64_t p0 = start; p0 < stop; p0 += kScopeWave) {
      const uint64_t p = p0 + lane;
      const bool ok = p < stop && prim::load4(reinterpret_cast<const uint8_t*>(a.lev + p)) <= lv;
      const uint64_t bm = prim::ballot(ok);
      if (bm) {
        found = (int64_t)(p0 + (uint64_t)__builtin_ctzll(bm));
        break;
      }
    }
    if (found >= 0 && lane == 0) resolve(a, i, (uint32_t)found, ki);
  }
}

JSIDX_DEV bool value_start(uint32_t t) { return t == kOther || t == kOpenSq || t == kOpenCu || t == kStr; }
JSIDX_DEV uint32_t tok_at(const ScopeArgs& a, int64_t i) { return i < 0 ? 0xFFu : prim::load1(a.kind + i); }
// A string at entry j is an object key: it follows '{' or a comma of an object.
JSIDX_DEV bool is_key(const ScopeArgs& a, int64_t j) {
  if (j < 1) return false;
  const uint32_t p = tok_at(a, j - 1);
  return p == kOpenCu || (p == kComma && prim::load1(a.ck + j - 1) == kCloseCu);
}

// Structure check of entry i: its token must be allowed after the one before
// it (a comma's successor by the comma's scope, a string's by whether it is a
// key), nothing may follow the root value, and the last entry must end it.
JSIDX_DEV void check_entry(const ScopeArgs& a, uint64_t i) {
  const uint32_t cur = tok_at(a, (int64_t)i);
  bool bad;
  if (i == 0) {
    bad = !value_start(cur);
  } else {
    const uint32_t p = tok_at(a, (int64_t)i - 1);
    const bool key_before = p == kStr && is_key(a, (int64_t)i - 1);
    if (p == kOpenCu) bad = !(cur == kStr || cur == kCloseCu);
    else if (p == kOpenSq) bad = !(value_start(cur) || cur == kCloseSq);
    else if (p == kColon) bad = !value_start(cur);
    else if (p == kComma) {
      const uint32_t s = prim::load1(a.ck + i - 1);
      bad = s == kCloseCu ? cur != kStr : (s == kCloseSq ? !value_start(cur) : true);
    } else if (key_before) {
      bad = cur != kColon;
    } else {  // after a value: a comma or a closer inside a scope, nothing at the root
      bad = prim::load4(reinterpret_cast<const uint8_t*>(a.dep + i)) == 0u ||
            !(cur == kComma || cur == kCloseSq || cur == kCloseCu);
    }
  }
  if (i + 1 == a.n) {  // the last entry ends the root value
    const bool ends = cur == kOther || cur == kCloseSq || cur == kCloseCu || (cur == kStr && !is_key(a, (int64_t)i));
    bad = bad || !ends;
  }
  if (bad) prim::or_agent32(a.err, kErrSyntax);
}

// 6. The structure check over all entries (a grid-stride loop).  With the
//    links unbalanced or mismatched the structure is invalid too.
JSIDX_DEVFN void scope_check(const ScopeArgs& a) {
  const uint64_t first = (uint64_t)prim::block() * kScopeThreads + scope_tid();
  if (first == 0 && (prim::ld_agent32(a.err) & (kErrUnbalanced | kErrMismatched)))
    prim::or_agent32(a.err, kErrSyntax);
  for (uint64_t i = first; i < a.n; i += (uint64_t)prim::grid() * kScopeThreads) check_entry(a, i);
}

}  // namespace jsidx
