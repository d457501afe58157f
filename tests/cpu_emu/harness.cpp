// Runs the indexing kernel body on the CPU through the emulated primitives --
// TEST INFRASTRUCTURE ONLY (see jsidx_prims.h next to this file).
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <thread>
#include <vector>

#include "jsidx_doc.h"
#include "jsidx_kernel.h"
#include "jsidx_scopes.h"
#include "jsidx_tape.h"

namespace jsidx {
namespace prim {
thread_local ThreadCtx tctx;
}
}  // namespace jsidx

using namespace jsidx;

extern "C" {

// Index through the kernel body with `nblocks` concurrent waves (rounded up
// to whole workgroups).
//   granule_lo/hi: the bytes the kernel may read (the aligned 16-byte granules
//   overlapping the input).  Returns the number of out-of-range accesses.
//   ws_state: persistent workspace (caller allocated, zeroed once) so that
//   several launches can reuse it like the real library does; cap_tiles
//   counts largest tiles.
//   rows: rows per tile (0: the kernel picks them for the launch's waves).
//   minify: run the minify pass (out_idx then receives bytes).
//   variant: the indexing kernel's variant (0 or one kVar* flag).
long emu_run(const uint8_t* base, const uint64_t* offsets, uint64_t len, uint32_t ndocs, uint32_t* out_idx,
             uint64_t out_cap, uint32_t* out_n, uint32_t* out_err, int nblocks, void* ws_mem, uint64_t cap_tiles,
             uint32_t rows, const uint8_t* granule_lo, const uint8_t* granule_hi, int minify, int variant) {
  prim::EmuEnv env;
  env.reads[env.nreads++] = {granule_lo, granule_hi};
  if (offsets) env.reads[env.nreads++] = {offsets, offsets + ndocs + 1};
  // out_cap counts entries: uint32 positions, or bytes when minifying
  env.writes[env.nwrites++] = {out_idx, reinterpret_cast<const uint8_t*>(out_idx) + out_cap * (minify ? 1 : 4)};
  env.writes[env.nwrites++] = {out_n, out_n + ndocs};
  env.writes[env.nwrites++] = {out_err, out_err + ndocs};
  env.writes[env.nwrites++] = {ws_mem, (const uint8_t*)ws_mem + stream_ws_bytes(cap_tiles)};
  env.reads[env.nreads++] = {ws_mem, (const uint8_t*)ws_mem + stream_ws_bytes(cap_tiles)};

  Args a;
  a.base = base;
  a.offsets = offsets;
  a.len = len;
  a.ndocs = ndocs;
  a.out_idx = out_idx;
  a.out_n = out_n;
  a.out_err = out_err;
  a.ws = (Workspace*)ws_mem;
  a.cap_tiles = desc_slots(cap_tiles);
  a.cap_rows = cap_tiles * (uint64_t)kRows;

  // a batch's offsets are checked first, as the library launches it
  if (offsets) {
    constexpr int kCheck = 128;
    std::vector<prim::GroupCtx*> cg;
    for (int b = 0; b < 2; b++) cg.push_back(new prim::GroupCtx(kCheck));
    std::vector<std::thread> ct;
    for (int b = 0; b < 2; b++) {
      for (uint32_t t = 0; t < (uint32_t)kCheck; t++) {
        ct.emplace_back([&, b, t] {
          prim::tctx.tid = t;
          prim::tctx.block = (uint32_t)b;
          prim::tctx.grid = 2;
          prim::tctx.g = cg[(size_t)b];
          prim::tctx.env = &env;
          offsets_check(offsets, ndocs, (Workspace*)ws_mem, kCheck);
        });
      }
    }
    for (auto& x : ct) x.join();
    for (auto* g : cg) delete g;
  }

  // nblocks counts waves; they run as whole workgroups of kWaves waves
  const int ngroups = (nblocks + kWaves - 1) / kWaves;
  a.rows = rows;
  a.fill_waves = (uint32_t)(ngroups * kWaves);
  for (int i = 0; i < 4; i++) a.rows_tab[i] = 0;
  std::vector<prim::GroupCtx*> groups;
  for (int b = 0; b < ngroups; b++) groups.push_back(new prim::GroupCtx(kGroupThreads));
  std::vector<std::thread> th;
  for (int b = 0; b < ngroups; b++) {
    for (uint32_t t = 0; t < (uint32_t)kGroupThreads; t++) {
      th.emplace_back([&, b, t] {
        prim::tctx.tid = t;
        prim::tctx.block = (uint32_t)b;
        prim::tctx.grid = (uint32_t)ngroups;
        prim::tctx.g = groups[(size_t)b];
        prim::tctx.env = &env;
        if (minify) index_tiles<true>(a);
        else if (variant == kVarNaiveClassify) index_tiles<false, kVarNaiveClassify>(a);
        else if (variant == kVarXorLoop) index_tiles<false, kVarXorLoop>(a);
        else if (variant == kVarDirectFlatten) index_tiles<false, kVarDirectFlatten>(a);
        else index_tiles<false>(a);
      });
    }
  }
  for (auto& x : th) x.join();
  for (auto* g : groups) delete g;
  return env.violations.load();
}

// The scope-link kernels, each run as a grid of workgroups of kScopeThreads
// threads, in launch order.  Returns the number of out-of-range accesses.
long emu_scopes_run(const uint8_t* buf, uint64_t len, const uint32_t* idx, uint32_t n, uint32_t* match,
                    uint32_t* err, void* ws, int far_groups) {
  const ScopeLayout L = scope_layout(n);
  prim::EmuEnv env;
  if (len) env.reads[env.nreads++] = {buf, buf + len};
  if (n) env.reads[env.nreads++] = {idx, idx + n};
  env.writes[env.nwrites++] = {match, match + n};
  env.writes[env.nwrites++] = {err, err + 1};
  env.writes[env.nwrites++] = {ws, (const uint8_t*)ws + L.total};
  env.reads[env.nreads++] = {ws, (const uint8_t*)ws + L.total};
  env.reads[env.nreads++] = {match, match + n};
  uint8_t* m = static_cast<uint8_t*>(ws);
  ScopeArgs a;
  a.buf = buf;
  a.len = len;
  a.idx = idx;
  a.n = n;
  a.nchunks = (uint32_t)((n + (uint64_t)kScopeChunk - 1) / kScopeChunk);
  a.match = match;
  a.err = err;
  a.chunk_fn = reinterpret_cast<uint2*>(m + L.chunk_fn);
  a.in_depth = reinterpret_cast<uint2*>(m + L.in_depth);
  a.chunk_min = reinterpret_cast<uint32_t*>(m + L.chunk_min);
  a.qcount = reinterpret_cast<uint32_t*>(m + L.qcount);
  a.lev = reinterpret_cast<uint32_t*>(m + L.lev);
  a.queue = reinterpret_cast<uint32_t*>(m + L.queue);
  a.kind = m + L.kind;
  auto phase = [&](int ngroups, void (*body)(const ScopeArgs&)) {
    std::vector<prim::GroupCtx*> groups;
    for (int b = 0; b < ngroups; b++) groups.push_back(new prim::GroupCtx(kScopeThreads));
    std::vector<std::thread> th;
    for (int b = 0; b < ngroups; b++) {
      for (uint32_t t = 0; t < (uint32_t)kScopeThreads; t++) {
        th.emplace_back([&, b, t] {
          prim::tctx.tid = t;
          prim::tctx.block = (uint32_t)b;
          prim::tctx.grid = (uint32_t)ngroups;
          prim::tctx.g = groups[(size_t)b];
          prim::tctx.env = &env;
          body(a);
        });
      }
    }
    for (auto& x : th) x.join();
    for (auto* g : groups) delete g;
  };
  if (a.nchunks) phase((int)a.nchunks, scope_chunk_fn<false>);
  phase(1, scope_scan<false>);
  if (a.nchunks) {
    phase((int)a.nchunks, scope_levels<false>);
    phase((int)a.nchunks, scope_local<false>);
    phase(far_groups, scope_far<false>);
    phase((int)a.nchunks, scope_check<false>);
  }
  return env.violations.load();
}

uint64_t emu_scopes_ws_bytes(uint64_t n) { return scope_layout(n).total; }
uint64_t emu_scopes_batch_ws_bytes(uint64_t cap, uint64_t ndocs) { return scope_batch_layout(cap, ndocs).total; }

// The batched scope kernels over ndocs documents (bytes at buf, offsets,
// index entries at idx + offsets[d], counts n[d]), with chunk_groups
// workgroups for the chunk kernels and doc_groups for the per-document ones.
long emu_scopes_batch_run(const uint8_t* buf, const uint64_t* offsets, uint32_t ndocs, const uint32_t* idx,
                          const uint32_t* n, uint32_t* match, uint32_t* err, void* ws, uint64_t cap, int chunk_groups,
                          int doc_groups, int far_groups) {
  const ScopeBatchLayout L = scope_batch_layout(cap, ndocs);
  const uint64_t total = offsets[ndocs];
  prim::EmuEnv env;
  if (total) env.reads[env.nreads++] = {buf, buf + total};
  env.reads[env.nreads++] = {offsets, offsets + ndocs + 1};
  if (total) env.reads[env.nreads++] = {idx, idx + total};
  env.reads[env.nreads++] = {n, n + ndocs};
  if (total) env.writes[env.nwrites++] = {match, match + total};
  env.writes[env.nwrites++] = {err, err + ndocs};
  env.writes[env.nwrites++] = {ws, (const uint8_t*)ws + L.total};
  env.reads[env.nreads++] = {ws, (const uint8_t*)ws + L.total};
  uint8_t* m = static_cast<uint8_t*>(ws);
  ScopeArgs a;
  a.buf = buf;
  a.len = 0;
  a.idx = idx;
  a.n = 0;
  a.nchunks = 0;
  a.match = reinterpret_cast<uint32_t*>(m + L.match);
  a.err = err;
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
  a.out_match = match;
  auto phase = [&](int ngroups, void (*body)(const ScopeArgs&)) {
    std::vector<prim::GroupCtx*> groups;
    for (int b = 0; b < ngroups; b++) groups.push_back(new prim::GroupCtx(kScopeThreads));
    std::vector<std::thread> th;
    for (int b = 0; b < ngroups; b++) {
      for (uint32_t t = 0; t < (uint32_t)kScopeThreads; t++) {
        th.emplace_back([&, b, t] {
          prim::tctx.tid = t;
          prim::tctx.block = (uint32_t)b;
          prim::tctx.grid = (uint32_t)ngroups;
          prim::tctx.g = groups[(size_t)b];
          prim::tctx.env = &env;
          body(a);
        });
      }
    }
    for (auto& x : th) x.join();
    for (auto* g : groups) delete g;
  };
  const int sg = (int)docscan_groups(ndocs);
  phase(sg, scope_batch_sums);
  phase(1, scope_batch_bases);
  phase(sg, scope_batch_starts);
  phase(doc_groups, scope_batch_compact);
  phase(chunk_groups, scope_chunk_fn<true>);
  phase(1, scope_scan<true>);
  phase(chunk_groups, scope_levels<true>);
  phase(chunk_groups, scope_local<true>);
  phase(far_groups, scope_far<true>);
  phase(chunk_groups, scope_check<true>);
  phase(doc_groups, scope_batch_finish);
  return env.violations.load();
}

// The tape kernels (jsidx_tape.h) over one document's index and links.
// Returns the number of out-of-range accesses.
long emu_tape_run(const uint8_t* buf, uint64_t len, const uint32_t* idx, uint32_t n, const uint32_t* match,
                  uint64_t* tape, uint64_t tape_cap, uint8_t* str, uint64_t str_cap, uint64_t* tape_n, uint64_t* str_n,
                  uint32_t* err, void* ws, int exact_groups, uint32_t* exact_count) {
  const TapeLayout L = tape_layout(n);
  prim::EmuEnv env;
  if (len) env.reads[env.nreads++] = {buf, buf + len};
  if (n) env.reads[env.nreads++] = {idx, idx + n};
  if (n) env.reads[env.nreads++] = {match, match + n};
  env.reads[env.nreads++] = {ws, (const uint8_t*)ws + L.total};
  env.writes[env.nwrites++] = {tape, tape + tape_cap};
  env.writes[env.nwrites++] = {str, str + str_cap};
  env.writes[env.nwrites++] = {tape_n, tape_n + 1};
  env.writes[env.nwrites++] = {str_n, str_n + 1};
  env.writes[env.nwrites++] = {err, err + 1};
  env.writes[env.nwrites++] = {ws, (const uint8_t*)ws + L.total};
  uint8_t* m = static_cast<uint8_t*>(ws);
  TapeArgs a;
  a.buf = buf;
  a.len = len;
  a.idx = idx;
  a.n = n;
  a.nchunks = (uint32_t)((n + (uint64_t)kTapeChunk - 1) / kTapeChunk);
  a.match = match;
  a.tape = tape;
  a.str = str;
  a.tape_n = tape_n;
  a.str_n = str_n;
  a.err = err;
  a.chunk_sum = reinterpret_cast<uint64_t*>(m + L.chunk_sum);
  a.sbytes = reinterpret_cast<uint32_t*>(m + L.sbytes);
  a.toff = reinterpret_cast<uint32_t*>(m + L.toff);
  a.kb = m + L.kb;
  a.runbad = m + L.runbad;
  a.qcount = reinterpret_cast<uint32_t*>(m + L.qcount);
  a.queue = reinterpret_cast<uint32_t*>(m + L.queue);
  a.nqueue = reinterpret_cast<uint2*>(m + L.nqueue);
  auto phase = [&](int ngroups, int nthreads, void (*body)(const TapeArgs&)) {
    std::vector<prim::GroupCtx*> groups;
    for (int b = 0; b < ngroups; b++) groups.push_back(new prim::GroupCtx((uint32_t)nthreads));
    std::vector<std::thread> th;
    for (int b = 0; b < ngroups; b++) {
      for (uint32_t t = 0; t < (uint32_t)nthreads; t++) {
        th.emplace_back([&, b, t] {
          prim::tctx.tid = t;
          prim::tctx.block = (uint32_t)b;
          prim::tctx.grid = (uint32_t)ngroups;
          prim::tctx.g = groups[(size_t)b];
          prim::tctx.env = &env;
          body(a);
        });
      }
    }
    for (auto& x : th) x.join();
    for (auto* g : groups) delete g;
  };
  if (a.nchunks) phase((int)a.nchunks, kTapeThreads, tape_count<false>);
  phase(1, kTapeThreads, tape_scan<false>);
  if (a.nchunks) {
    phase((int)a.nchunks, kTapeThreads, tape_offsets<false>);
    phase((int)a.nchunks, kTapeThreads, tape_write<false>);
    phase(2, kTapeThreads, tape_numbers<false>);
    phase(exact_groups, kExactThreads, tape_exact<false>);
  }
  *exact_count = n ? *a.qcount : 0u;
  return env.violations.load();
}

uint64_t emu_tape_ws_bytes(uint64_t n) { return tape_layout(n).total; }
// Where the workspace records which runs left their strings to the per-string path.
uint64_t emu_tape_runbad_offset(uint64_t n) { return tape_layout(n).runbad; }
uint64_t emu_tape_batch_runbad_offset(uint64_t cap, uint64_t ndocs) { return tape_batch_layout(cap, ndocs).runbad; }
uint64_t emu_tape_batch_ws_bytes(uint64_t cap, uint64_t ndocs) { return tape_batch_layout(cap, ndocs).total; }

// The batched tape kernels over ndocs documents (index and links in the
// batch layout); out_pos receives each document's tape start and words,
// string start and bytes.  Returns the number of out-of-range accesses.
long emu_tape_batch_run(const uint8_t* buf, const uint64_t* offsets, uint32_t ndocs, const uint32_t* idx,
                        const uint32_t* n, const uint32_t* match, uint64_t* tape, uint64_t tape_cap, uint8_t* str,
                        uint64_t str_cap, uint64_t* out_pos, uint32_t* err, void* ws, uint64_t cap, int chunk_groups,
                        int doc_groups, int exact_groups) {
  const TapeBatchLayout L = tape_batch_layout(cap, ndocs);
  const uint64_t total = offsets[ndocs];
  prim::EmuEnv env;
  if (total) env.reads[env.nreads++] = {buf, buf + total};
  env.reads[env.nreads++] = {offsets, offsets + ndocs + 1};
  if (total) env.reads[env.nreads++] = {idx, idx + total};
  if (total) env.reads[env.nreads++] = {match, match + total};
  env.reads[env.nreads++] = {n, n + ndocs};
  env.reads[env.nreads++] = {ws, (const uint8_t*)ws + L.total};
  env.writes[env.nwrites++] = {tape, tape + tape_cap};
  env.writes[env.nwrites++] = {str, str + str_cap};
  env.writes[env.nwrites++] = {out_pos, out_pos + 4 * (uint64_t)ndocs};
  env.writes[env.nwrites++] = {err, err + ndocs};
  env.writes[env.nwrites++] = {ws, (const uint8_t*)ws + L.total};
  uint8_t* m = static_cast<uint8_t*>(ws);
  TapeArgs a{};
  a.buf = buf;
  a.idx = idx;
  a.match = match;
  a.tape = tape;
  a.str = str;
  a.err = err;
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
  auto phase = [&](int ngroups, int nthreads, void (*body)(const TapeArgs&)) {
    std::vector<prim::GroupCtx*> groups;
    for (int b = 0; b < ngroups; b++) groups.push_back(new prim::GroupCtx((uint32_t)nthreads));
    std::vector<std::thread> th;
    for (int b = 0; b < ngroups; b++) {
      for (uint32_t t = 0; t < (uint32_t)nthreads; t++) {
        th.emplace_back([&, b, t] {
          prim::tctx.tid = t;
          prim::tctx.block = (uint32_t)b;
          prim::tctx.grid = (uint32_t)ngroups;
          prim::tctx.g = groups[(size_t)b];
          prim::tctx.env = &env;
          body(a);
        });
      }
    }
    for (auto& x : th) x.join();
    for (auto* g : groups) delete g;
  };
  const int sg = (int)docscan_groups(ndocs);
  phase(sg, kTapeThreads, tape_batch_sums);
  phase(1, kTapeThreads, tape_batch_bases);
  phase(sg, kTapeThreads, tape_batch_starts);
  phase(doc_groups, kTapeThreads, tape_batch_compact);
  phase(chunk_groups, kTapeThreads, tape_count<true>);
  phase(1, kTapeThreads, tape_scan<true>);
  phase(chunk_groups, kTapeThreads, tape_offsets<true>);
  phase(doc_groups, kTapeThreads, tape_batch_docs);
  phase(chunk_groups, kTapeThreads, tape_write<true>);
  phase(2, kTapeThreads, tape_numbers<true>);
  phase(exact_groups, kExactThreads, tape_exact<true>);
  return env.violations.load();
}

// One number text through the fast conversion (exact == 0; the grammar scan
// first) or the exact one (exact == 1).  Returns kConvOk / kConvInf /
// kConvUndecided (-1: the grammar rejects it), the magnitude's bits in *bits.
int emu_number(const uint8_t* text, uint64_t len, int exact, uint64_t* bits) {
  prim::EmuEnv env;
  env.reads[env.nreads++] = {text, text + len};
  prim::GroupCtx g(1);
  prim::tctx.tid = 0;
  prim::tctx.block = 0;
  prim::tctx.grid = 1;
  prim::tctx.g = &g;
  prim::tctx.env = &env;
  TapeArgs a{};
  a.buf = text;
  a.len = len;
  const NumText t = scan_number(a, 0);
  if (!t.ok) return -1;
  *bits = 0;
  if (exact) {
    static thread_local ExactScratch x;
    return exact_double(a, 0, x.D, x.V, x.S, bits);
  }
  if (t.w == 0) return kConvOk;
  int r = fast_double(t.w, t.q, bits);
  if (r != kConvUndecided && t.trunc) {
    uint64_t b2 = 0;
    const int r2 = fast_double(t.w + 1, t.q, &b2);
    if (r2 != r || (r == kConvOk && b2 != *bits)) r = kConvUndecided;
  }
  return r;
}

uint64_t emu_ws_bytes(uint64_t cap_tiles) { return stream_ws_bytes(cap_tiles); }

// One document through the one-document kernel (jsidx_doc.h) with `nwaves`
// concurrent waves (rounded up to whole workgroups), over the persistent
// workspace ws_mem of cap_tiles largest tiles.  granule_lo/hi: the bytes the
// kernel may read.  Returns the number of out-of-range accesses.
long emu_doc_run(const uint8_t* base, uint64_t len, uint32_t* out_idx, uint64_t out_cap, uint32_t* out_n,
                 uint32_t* out_err, int nwaves, void* ws_mem, uint64_t cap_tiles, const uint8_t* granule_lo,
                 const uint8_t* granule_hi, int variant) {
  prim::EmuEnv env;
  env.reads[env.nreads++] = {granule_lo, granule_hi};
  env.writes[env.nwrites++] = {out_idx, out_idx + out_cap};
  env.writes[env.nwrites++] = {out_n, out_n + 1};
  env.writes[env.nwrites++] = {out_err, out_err + 1};
  env.writes[env.nwrites++] = {ws_mem, (const uint8_t*)ws_mem + stream_ws_bytes(cap_tiles)};
  env.reads[env.nreads++] = {ws_mem, (const uint8_t*)ws_mem + stream_ws_bytes(cap_tiles)};
  DocArgs a;
  a.base = base;
  a.len = len;
  a.out_idx = out_idx;
  a.out_n = out_n;
  a.out_err = out_err;
  a.ws = (Workspace*)ws_mem;
  uint8_t* region = (uint8_t*)ws_mem + doc_region_offset(cap_tiles);
  a.cap = doc_cap_for(cap_tiles);
  a.desc = (uint64_t*)region;
  a.blk = a.desc + a.cap;
  a.bcnt = (uint32_t*)(a.blk + 2 * doc_blocks_for(a.cap));
  a.p0 = -(int64_t)((uintptr_t)base & 15u);
  a.ntiles = len ? ((int64_t)len - a.p0 + kDocTile - 1) / kDocTile : 0;
  const int ngroups = (nwaves + kDocWaves - 1) / kDocWaves;
  std::vector<prim::GroupCtx*> groups;
  for (int b = 0; b < ngroups; b++) groups.push_back(new prim::GroupCtx(kDocThreads));
  std::vector<std::thread> th;
  for (int b = 0; b < ngroups; b++) {
    for (uint32_t t = 0; t < (uint32_t)kDocThreads; t++) {
      th.emplace_back([&, b, t] {
        prim::tctx.tid = t;
        prim::tctx.block = (uint32_t)b;
        prim::tctx.grid = (uint32_t)ngroups;
        prim::tctx.g = groups[(size_t)b];
        prim::tctx.env = &env;
        if (variant == kVarNaiveClassify) doc_tiles<kVarNaiveClassify>(a);
        else if (variant == kVarXorLoop) doc_tiles<kVarXorLoop>(a);
        else if (variant == kVarDirectFlatten) doc_tiles<kVarDirectFlatten>(a);
        else doc_tiles<0>(a);
      });
    }
  }
  for (auto& x : th) x.join();
  for (auto* g : groups) delete g;
  return env.violations.load();
}
uint32_t emu_doc_tile_bytes() { return (uint32_t)kDocTile; }
uint32_t emu_doc_slots() { return (uint32_t)kDocSlots; }
uint32_t emu_tile_bytes() { return (uint32_t)kTileBytes; }
uint32_t emu_pick_rows(int64_t span, uint64_t waves) { return pick_rows(span, waves); }

}  // extern "C"
