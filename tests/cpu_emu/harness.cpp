// Runs the indexing kernel body on the CPU through the emulated primitives --
// TEST INFRASTRUCTURE ONLY (see jsidx_prims.h next to this file).
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <thread>
#include <vector>

#include "jsidx_kernel.h"

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
long emu_run(const uint8_t* base, const uint64_t* offsets, uint64_t len, uint32_t ndocs, uint32_t* out_idx,
             uint64_t out_cap, uint32_t* out_n, uint32_t* out_err, int nblocks, void* ws_mem, uint64_t cap_tiles,
             uint32_t rows, const uint8_t* granule_lo, const uint8_t* granule_hi, int minify) {
  prim::EmuEnv env;
  env.reads[env.nreads++] = {granule_lo, granule_hi};
  if (offsets) env.reads[env.nreads++] = {offsets, offsets + ndocs + 1};
  // out_cap counts entries: uint32 positions, or bytes when minifying
  env.writes[env.nwrites++] = {out_idx, reinterpret_cast<const uint8_t*>(out_idx) + out_cap * (minify ? 1 : 4)};
  env.writes[env.nwrites++] = {out_n, out_n + ndocs};
  env.writes[env.nwrites++] = {out_err, out_err + ndocs};
  env.writes[env.nwrites++] = {ws_mem, (const uint8_t*)ws_mem + workspace_bytes(cap_tiles)};
  env.reads[env.nreads++] = {ws_mem, (const uint8_t*)ws_mem + workspace_bytes(cap_tiles)};

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
        if (minify) index_tiles<true>(a); else index_tiles<false>(a);
      });
    }
  }
  for (auto& x : th) x.join();
  for (auto* g : groups) delete g;
  return env.violations.load();
}

uint64_t emu_ws_bytes(uint64_t cap_tiles) { return workspace_bytes(cap_tiles); }
uint32_t emu_tile_bytes() { return (uint32_t)kTileBytes; }
uint32_t emu_pick_rows(int64_t span, uint64_t waves) { return pick_rows(span, waves); }

}  // extern "C"
