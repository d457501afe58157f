// jsidx_kernel.h -- the stage-1 indexing kernel body (see jsidx.hip for the
// design summary).  Written against the primitives of jsidx_prims.h only.
//
// One wave is one workgroup and owns one tile of kTileBytes at a time: kRows
// rows of 64 lanes x 32 bytes, processed one row after the other.  All carries
// inside a tile (escape, in-string, predecessor, UTF-8 error, counts) move
// between lanes by wave ballots and between rows in scalar registers, so a
// tile needs no workgroup barrier.  Carries between tiles use a single
// decoupled look-back per tile.  Because a tile's result depends on whether it
// starts inside a string, each tile keeps two masks per row: K, the bytes that
// are candidates (structural, quote, or a pseudo-structural candidate), and
// F0, the indexed bytes assuming the tile does not start inside a string.  If
// it does, the indexed bytes of the region before the tile's first document
// start are F0 ^ K (every candidate flips: Sec. 3.1.3's formulas are symmetric
// in R), so the look-back only has to deliver the incoming state.  Bytes at or
// after the first document start never depend on the incoming state; they are
// written during the local pass, before the look-back.
#pragma once
#include <stdint.h>

#include "jsidx.h"
#include "jsidx_device.h"

namespace jsidx {

constexpr int kThreads = 64;  // lanes per wave; a wave owns one tile at a time
// Waves per workgroup (they share only their first tickets); tuning builds
// may override.
#ifndef JSIDX_GROUP_WAVES
#define JSIDX_GROUP_WAVES 8
#endif
constexpr int kWaves = JSIDX_GROUP_WAVES;
constexpr int kGroupThreads = kWaves * kThreads;
// Consecutive tiles per ticket (when every wave gets at least that many).
// A wave finishes a tile after starting the next, so with two tiles per
// ticket both are published before the wave first waits.  With more, a
// ticket's later tiles would be published only after the wave waited on
// earlier tiles, whose owners wait in turn: a chain through every wave.
#ifndef JSIDX_TICKET_TILES
#define JSIDX_TICKET_TILES 2
#endif
constexpr int kTicketTiles = JSIDX_TICKET_TILES;
static_assert(kTicketTiles == 1 || kTicketTiles == 2, "a ticket's tiles must all publish before its wave waits");
constexpr int kSegBytes = 32;
constexpr int kRowBytes = kThreads * kSegBytes;  // 2 KiB
// Rows per tile: at most kRows (tuning builds may override), at least
// kMinRows.  Each launch picks its tile size (see pick_rows).
#ifndef JSIDX_TILE_ROWS
#define JSIDX_TILE_ROWS 16
#endif
constexpr int kRows = JSIDX_TILE_ROWS;
constexpr int kMinRows = 2;
constexpr int kTileBytes = kRows * kRowBytes;  // largest tile: 32 KiB
static_assert(kRows >= kMinRows && kRows % kMinRows == 0 && (kRows & (kRows - 1)) == 0, "tile rows");
constexpr int kDocCap = 256;                   // documents per tile held in LDS
constexpr int kScrub = 4096;                   // descriptors cleared per launch
constexpr int kEscSteps = 4;                   // backslash run scanned back: 4 x 1 KiB
// Rows of input in flight ahead of the row being classified.
#ifndef JSIDX_PREFETCH_ROWS
#define JSIDX_PREFETCH_ROWS 1
#endif
// Flatten through LDS: a row's positions are gathered in LDS and written out
// with coalesced stores (rows of at most kStage positions).
#ifndef JSIDX_STAGED_FLATTEN
#define JSIDX_STAGED_FLATTEN 1
#endif
constexpr int kStage = 512;
// Variants of the indexing kernel, each turning one of the paper's stage-1
// optimizations off (the ablation of App. B, Table of optimizations, replayed):
//   kVarNaiveClassify: classes by one comparison per class character and byte,
//                      ORed, instead of nibble logic on bit planes;
//   kVarXorLoop:       the in-string mask by toggling from each quote upward,
//                      one step per quote, instead of the shift/XOR ladder;
//   kVarDirectFlatten: every lane stores its own positions, the paper's naive
//                      trailing-zero loop, instead of staging dense rows in LDS.
constexpr int kVarNaiveClassify = 1;
constexpr int kVarXorLoop = 2;
constexpr int kVarDirectFlatten = 4;
#ifndef JSIDX_STAGE_LANE
#define JSIDX_STAGE_LANE 8
#endif
// Tiles per look-back block (at most 4 per lane); test builds shrink it to
// reach many blocks with small inputs.
#ifndef JSIDX_BLOCK_TILES
#define JSIDX_BLOCK_TILES 256
#endif
constexpr int kBlockTiles = JSIDX_BLOCK_TILES;
static_assert(kBlockTiles >= 1 && kBlockTiles <= 256, "a block must fit one look-back window");
static_assert(kTileBytes < 65536, "tile counts must fit in 16 bits");

// ---- tile descriptors for the look-back ----------------------------------
// bits 0..1 flag, 2..43 payload, 44..63 launch epoch.
//   aggregate: 2..9 transfer table, 10..25 count if the tile starts outside a
//              string, 26..41 count if inside, 42 byte 0 is a pseudo-structural
//              candidate, 43 the tile's counts depend on the incoming escape
//   inclusive: 2..5 state after the tile, 6 a document starts in the tile,
//              7..38 count of the current document up to the tile's end
enum : uint32_t { kNone = 0, kAgg = 1, kInc = 2 };
constexpr uint32_t kEpochShift = 44;
constexpr uint64_t kEpochMask = (1ull << 20) - 1;

// Workspace: this header, then cap_tiles tile descriptors, 3 words per block
// of block descriptors, one 32-bit counter per block, and the head-region
// masks of every tile.  A workspace is sized in largest tiles (tiles16); it
// holds a descriptor for every smallest tile of that many bytes.
struct Workspace {
  uint32_t ticket;  // next tile to hand out
  uint32_t done;    // workgroups that have left the tile loop
  uint32_t epoch;   // launch counter (tags descriptors)
  uint32_t diag;    // sticky: 1 = a look-back wait gave up (never expected)
  uint32_t bad;     // set by offsets_check when a batch's offsets decrease;
                    // cleared by the last workgroup of the launch after it
  uint32_t pad;
  uint64_t desc[1];  // one per tile
};

inline constexpr uint64_t blocks_for_tiles(uint64_t tiles) { return (tiles + kBlockTiles - 1) / kBlockTiles; }
// Head-region masks of a tile (candidates, indexed bits if the tile starts
// outside a string): one pair per lane and row.
constexpr uint64_t kMaskBytesPerTile = (uint64_t)kRows * kThreads * 8;
inline constexpr uint64_t desc_slots(uint64_t tiles16) { return tiles16 * (uint64_t)(kRows / kMinRows); }
inline constexpr uint64_t mask_offset(uint64_t slots) {
  return (sizeof(Workspace) + slots * sizeof(uint64_t) + blocks_for_tiles(slots) * (3 * sizeof(uint64_t) + sizeof(uint32_t)) +
          255) & ~(uint64_t)255;
}
inline constexpr uint64_t workspace_bytes(uint64_t tiles16) {
  return mask_offset(desc_slots(tiles16)) + tiles16 * kMaskBytesPerTile;
}
// Rows per tile for a launch over `span` bytes with `waves` waves, unless
// tuned: the largest tile that still makes a tile for every eighth wave
// (small inputs get small tiles, so that more waves share them and a tile's
// serial chain of rows is short; past that, larger tiles cost less per
// byte), never below kMinRows.
inline constexpr uint32_t pick_rows(int64_t span, uint64_t waves) {
  uint32_t r = (uint32_t)kRows;
  const uint64_t target = waves / 8 ? waves / 8 : 1;
  while (r > (uint32_t)kMinRows && (uint64_t)(span > 0 ? span : 0) < (uint64_t)r * kRowBytes * target) r >>= 1;
  return r;
}
// Rows per tile from a tuning table: 4 bits per size class b =
// floor(log2(span)) (b = 0 for span <= 1), 0 = pick_rows, else rows = 1 << code.
inline constexpr uint32_t rows_for(int64_t span, uint64_t waves, const uint64_t* tab) {
  const uint32_t b = span > 1 ? 63u - (uint32_t)__builtin_clzll((uint64_t)span) : 0u;
  const uint32_t code = (uint32_t)(tab[b >> 4] >> (4u * (b & 15u))) & 15u;
  return code ? (1u << code) : pick_rows(span, waves);
}

JSIDX_DEV uint64_t epoch_bits(uint32_t epoch) { return ((uint64_t)epoch & kEpochMask) << kEpochShift; }
JSIDX_DEV uint64_t make_agg(uint32_t table, uint32_t c0, uint32_t c1, uint32_t elig0, uint32_t esens, uint32_t epoch) {
  return (uint64_t)kAgg | ((uint64_t)(table & 0xFFu) << 2) | ((uint64_t)(c0 & 0xFFFFu) << 10) |
         ((uint64_t)(c1 & 0xFFFFu) << 26) | ((uint64_t)(elig0 & 1u) << 42) | ((uint64_t)(esens & 1u) << 43) |
         epoch_bits(epoch);
}
JSIDX_DEV uint64_t make_inc(uint32_t state, uint32_t reset, uint32_t count, uint32_t epoch) {
  return (uint64_t)kInc | ((uint64_t)(state & 0xFu) << 2) | ((uint64_t)(reset & 1u) << 6) | ((uint64_t)count << 7) |
         epoch_bits(epoch);
}
JSIDX_DEV uint32_t d_flag(uint64_t d) { return (uint32_t)(d & 3u); }
JSIDX_DEV bool d_current(uint64_t d, uint32_t epoch) { return (d >> kEpochShift) == ((uint64_t)epoch & kEpochMask); }
JSIDX_DEV uint32_t d_table(uint64_t d) { return (uint32_t)(d >> 2) & 0xFFu; }
JSIDX_DEV uint32_t d_c0(uint64_t d) { return (uint32_t)(d >> 10) & 0xFFFFu; }
JSIDX_DEV uint32_t d_c1(uint64_t d) { return (uint32_t)(d >> 26) & 0xFFFFu; }
JSIDX_DEV uint32_t d_elig0(uint64_t d) { return (uint32_t)(d >> 42) & 1u; }
JSIDX_DEV uint32_t d_esens(uint64_t d) { return (uint32_t)(d >> 43) & 1u; }
JSIDX_DEV uint32_t d_state(uint64_t d) { return (uint32_t)(d >> 2) & 0xFu; }
JSIDX_DEV uint32_t d_reset(uint64_t d) { return (uint32_t)(d >> 6) & 1u; }
JSIDX_DEV uint32_t d_count(uint64_t d) { return (uint32_t)(d >> 7); }

JSIDX_DEV uint64_t ld_desc(Workspace* ws, int64_t j) { return prim::ld_agent(&ws->desc[j]); }
JSIDX_DEV void st_desc(Workspace* ws, int64_t j, uint64_t v) { prim::st_agent(&ws->desc[j], v); }

// ---- carry state between tiles ---------------------------------------------
// state bits: 0 e (next byte escaped), 1 q (inside a string), 2 p (previous
// byte structural/white space/quote), 3 u (UTF-8 error seen in this document).
// A tile's transfer (8 bits): bit 0 reset (a document starts in the tile),
// bit 1 u, bits 2..4 (e,q,p) out for e_in = 0, bits 5..7 for e_in = 1.  With
// reset, q and u are absolute; without, q is a flip and u is ORed.  p never
// depends on the incoming state (the tile is not empty).
JSIDX_DEV uint32_t tab_apply(uint32_t T, uint32_t s) {
  uint32_t e = s & 1u, q = (s >> 1) & 1u, u = (s >> 3) & 1u;
  uint32_t ent = (T >> (2 + 3 * e)) & 7u;
  uint32_t e2 = ent & 1u, q2 = (ent >> 1) & 1u, p2 = (ent >> 2) & 1u;
  uint32_t reset = T & 1u, tu = (T >> 1) & 1u;
  uint32_t qn = reset ? q2 : (q ^ q2);
  uint32_t un = reset ? tu : (u | tu);
  return e2 | (qn << 1) | (p2 << 2) | (un << 3);
}

struct Args {
  const uint8_t* base;      // bufs
  const uint64_t* offsets;  // null: one document [0, len)
  uint64_t len;
  uint32_t ndocs;
  uint32_t* out_idx;
  uint32_t* out_n;
  uint32_t* out_err;
  Workspace* ws;
  uint64_t cap_tiles;   // descriptors available (tiles of kMinRows rows)
  uint64_t cap_rows;    // rows of head-region masks available
  uint32_t rows;        // rows per tile (0: the kernel picks them)
  uint32_t fill_waves;  // waves of the launch (for picking rows)
  uint64_t rows_tab[4];  // tuning table of rows_for
};



JSIDX_DEV int64_t doc_off(const Args& a, int64_t d) {
  if (a.offsets) return (int64_t)prim::load8(a.offsets + d);
  return d <= 0 ? 0 : (int64_t)a.len;
}

// Per-wave LDS.
struct Shared {
  int64_t d_first;
  int64_t first_off;
  int32_t ntab;
  int32_t overflow;
  int32_t tab[kDocCap + 1];
  // indexed bits of plain rows after a document start, written after the
  // tile has published (the head region's masks live in the workspace)
  uint32_t hF[kRows][kThreads];
  // the head document ends in the head region: its last byte and flags there
  uint32_t he_valid, he_R0, he_EA, he_u;
  // plain rows after a document start, written after publishing: the
  // document's start and its count before the row
  int64_t tr_doff[kRows];
  uint32_t tr_cc[kRows];
#if JSIDX_STAGED_FLATTEN
  uint32_t stage[kStage];  // one row's positions on their way out
#endif
};

struct GroupShared {
  Shared w[kWaves];
  uint32_t first;    // the workgroup's first ticket
  uint32_t is_last;  // this workgroup finishes the launch
};

// Facts about a tile computed by tile_local (wave-uniform unless noted).
struct TileFacts {
  uint32_t carry;      // state after the tile
  uint32_t any_const;  // some byte is not a backslash or a document starts
  uint32_t lead_pos;   // first byte that is not a backslash or starts a doc
  uint32_t lead_reset; // ... and it is a document start
  uint32_t qsens;      // ... and it is a quote (its escape depends on e_in)
  uint32_t reset_any;
  uint32_t r0;         // first document start (kTileBytes: none)
  uint32_t elig0;      // byte 0 is a pseudo-structural candidate if p_in
  uint32_t head_rows;  // rows holding head-region bytes
  uint32_t a0, a1;     // per lane, head region: popcount(F0), popcount(K & ~F0)
  uint32_t tail_count; // count of the document open at the tile's end, since
                       // its start in this tile (valid if reset_any)
  uint32_t tail_rows;  // plain rows after a document start kept for writing
                       // after the tile has published (bit r = row r)
};

// Local document index of tile-relative position rel (table mode only): the
// last document starting at or before it (empty documents there come first).
JSIDX_DEVFN int32_t local_doc_of(const Shared& sh, int32_t rel) {
  int32_t lo = 0, hi = sh.ntab;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (sh.tab[mid] <= rel) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

JSIDX_DEVFN int64_t global_upper(const Args& a, int64_t lo, int64_t hi, int64_t pos) {
  // first d in [lo, hi) with doc_off(d) > pos; hi if none
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (doc_off(a, mid) <= pos) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Document (local index) holding tile-relative position rel, and its offset.
JSIDX_DEV int32_t doc_at(const Args& a, const Shared& sh, int64_t P0, int64_t d_first, int32_t rel) {
  if (!sh.overflow) return local_doc_of(sh, rel);
  return (int32_t)(global_upper(a, d_first, (int64_t)a.ndocs + 1, P0 + rel) - 1 - d_first);
}
JSIDX_DEV int64_t doc_start(const Args& a, const Shared& sh, int64_t P0, int64_t d_first, int32_t dloc) {
  if (dloc == 0) return sh.first_off;
  return !sh.overflow ? (int64_t)sh.tab[dloc] + P0 : doc_off(a, d_first + dloc);
}

JSIDX_DEV uint64_t lt_lanes() {
  uint32_t l = prim::lane();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}
JSIDX_DEV uint64_t lanes_below(int k) { return k <= 0 ? 0ull : (k >= 64 ? ~0ull : (~0ull >> (64 - k))); }
JSIDX_DEV int msb64(uint64_t m) { return 63 - __builtin_clzll(m); }
JSIDX_DEV uint32_t parity64(uint64_t m) { return (uint32_t)__builtin_popcountll(m) & 1u; }

// Lanes [k, lane) where k is the last lane below this one with `reset` set;
// all lanes below if none.  *from_carry: no such lane (the row carry applies).
JSIDX_DEV uint64_t span_since_reset(uint64_t resets, bool* from_carry) {
  uint64_t lt = lt_lanes();
  uint64_t m = resets & lt;
  *from_carry = (m == 0);
  if (!m) return lt;
  return lt & ~lanes_below(msb64(m));
}
// Lanes from the last reset lane (inclusive) to 63; all lanes if none.
JSIDX_DEV uint64_t tail_lanes(uint64_t resets) {
  if (!resets) return ~0ull;
  return ~lanes_below(msb64(resets));
}

JSIDX_DEV uint32_t wave_sum(uint32_t v) { return prim::readlane(prim::incl_scan(v), 63); }

// Segmented exclusive prefix of per-lane counts cv over the row: a lane with
// a document start (bit set in Rs) restarts the sum after it.  Returns the
// rank base of this lane's first piece (the one continuing from lanes below);
// *cc (uniform) is the count carried into the row and becomes the carry out.
JSIDX_DEV uint32_t row_ranks(uint32_t cv, uint64_t Rs, uint32_t* cc) {
  const uint32_t S = prim::incl_scan(cv);
  const uint32_t Sx = S - cv;  // sum over the lanes below
  // The last reset lane below has the largest exclusive sum among the reset
  // lanes below (+1 so that a sum of 0 still marks it).
  const uint32_t Mi = prim::incl_max_scan(prim::lane_bit(Rs) ? Sx + 1u : 0u);
  const uint32_t Me = prim::shr1(Mi, 0u);
  const uint32_t cin = Me ? Sx - (Me - 1u) : Sx + *cc;
  const uint32_t tot = prim::readlane(S, 63);
  if (Rs) *cc = tot - prim::readlane(Sx, msb64(Rs));
  else *cc += tot;
  return cin;
}

// This lane's 32 bytes at pos.  Only granules overlapping [begin, end) may be
// read: a granule outside is read from the granule holding byte `begin`
// instead, and its bytes are masked out by the caller's valid-byte mask.  The
// loads are unconditional, so no register write races a load in flight.
template <bool INTERIOR>
JSIDX_DEV void load_segment(const Args& a, int64_t pos, int64_t begin, int64_t end, uint32_t w[8]) {
  if (!INTERIOR && begin >= end) {  // empty input: nothing may be read
#pragma unroll
    for (int k = 0; k < 8; k++) w[k] = 0u;
    return;
  }
  const uint8_t* safe = reinterpret_cast<const uint8_t*>((reinterpret_cast<uintptr_t>(a.base) + (uintptr_t)begin) & ~(uintptr_t)15);
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int64_t g = pos + 16 * h;  // 16-byte aligned
    const bool ok = INTERIOR || (g < end && g + 16 > begin);
    const uint4 v = prim::load16(ok ? a.base + g : safe);
    w[4 * h + 0] = v.x; w[4 * h + 1] = v.y; w[4 * h + 2] = v.z; w[4 * h + 3] = v.w;
  }
}

// Writes the positions of this lane's set bits of F (the lane's 32 bytes start
// at document offset rel) at ranks from *cc plus the lanes below; *cc
// advances by the row's total.  Ranks at or past lim are not written (only a
// look-back that gave up could produce them).
template <bool STAGED = true>
JSIDX_DEV void write_row(Shared& sh, uint32_t* out, uint64_t lim, uint32_t* cc, uint32_t F, uint32_t rel) {
  const uint32_t n = (uint32_t)__builtin_popcount(F);
  const uint32_t incl = prim::incl_scan(n);
  const uint32_t row_n = prim::readlane(incl, 63);
  uint32_t kk = *cc + incl - n;
  const bool checked = (uint64_t)*cc + row_n > lim;
#if JSIDX_STAGED_FLATTEN
  // Direct writes take as many store instructions as the busiest lane has
  // positions, each touching several cache lines; through LDS they take one
  // coalesced store per 64 positions.  Rows where some lane holds more than
  // JSIDX_STAGE_LANE positions go through LDS.
  if (STAGED && !checked && row_n <= (uint32_t)kStage && prim::ballot(n > (uint32_t)JSIDX_STAGE_LANE) != 0ull) {
    // each lane puts its positions at their ranks in LDS, then the wave
    // writes the row's positions out as consecutive words
    uint32_t k = incl - n;
    while (F) {
      const uint32_t j = (uint32_t)__builtin_ctz(F);
      F &= F - 1u;
      sh.stage[k++] = rel + j;
    }
    prim::wave_sync();
    const uint32_t base = *cc;
    for (uint32_t i = prim::lane(); i < row_n; i += (uint32_t)kThreads) prim::st_out(out + base + i, sh.stage[i]);
    prim::wave_sync();  // the next row reuses the buffer
    *cc += row_n;
    return;
  }
#endif
  *cc += row_n;
  if (!checked) {
    while (F) {
      const uint32_t j = (uint32_t)__builtin_ctz(F);
      F &= F - 1u;
      prim::st_out(out + kk, rel + j);
      kk++;
    }
  } else {
    while (F) {
      const uint32_t j = (uint32_t)__builtin_ctz(F);
      F &= F - 1u;
      if ((uint64_t)kk < lim) prim::st_out(out + kk, rel + j);
      kk++;
    }
  }
}

// Byte J of a lane's 32-byte segment (J a compile-time constant, so that no
// register array is indexed at run time).
template <int J>
JSIDX_DEV uint32_t seg_byte(const uint32_t w[8]) { return (w[J >> 2] >> (8 * (J & 3))) & 0xFFu; }

// The bytes of F, in order, to dst[*k ...] (global memory, ranks below lim
// only) or, with TO_LDS, to the wave's LDS staging buffer.
template <int J, bool TO_LDS>
JSIDX_DEV void put_kept(uint8_t* dst, uint32_t F, const uint32_t w[8], uint32_t* k, uint32_t lim) {
  if ((F >> J) & 1u) {
    if constexpr (TO_LDS) dst[*k] = (uint8_t)seg_byte<J>(w);
    else if (*k < lim) prim::st_byte(dst + *k, seg_byte<J>(w));
    ++*k;
  }
  if constexpr (J < 31) put_kept<J + 1, TO_LDS>(dst, F, w, k, lim);
}

// Minified output of one row: the bytes of F (this lane's kept bytes, w its
// segment) at ranks from *cc plus the lanes below; *cc advances by the row's
// total.  The row's bytes are gathered in LDS at their ranks and written out
// with one store per 64 consecutive bytes.  Ranks at or past lim are not
// written.
JSIDX_DEV void write_bytes(Shared& sh, uint8_t* out, uint64_t lim, uint32_t* cc, uint32_t F, const uint32_t w[8]) {
  const uint32_t n = (uint32_t)__builtin_popcount(F);
  const uint32_t incl = prim::incl_scan(n);
  const uint32_t row_n = prim::readlane(incl, 63);
  const uint32_t base = *cc;
  *cc += row_n;
  if ((uint64_t)base + row_n <= lim) {
    uint8_t* sb = reinterpret_cast<uint8_t*>(sh.stage);  // 4 * kStage >= kRowBytes bytes
    uint32_t k = incl - n;
    put_kept<0, true>(sb, F, w, &k, 0xFFFFFFFFu);
    prim::wave_sync();
    for (uint32_t i = prim::lane(); i < row_n; i += (uint32_t)kThreads) prim::st_byte(out + base + i, sb[i]);
    prim::wave_sync();  // the next row reuses the buffer
  } else {
    uint32_t k = base + incl - n;
    put_kept<0, false>(out, F, w, &k, lim > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)lim);
  }
}

// ---------------------------------------------------------------------------
// The local pass over one tile, given the incoming state st_in.  Bytes at or
// after the tile's first document start do not depend on st_in: their
// positions and per-document results are written here.  Bytes before it (the
// head region) are written here too if `defer` is false (st_in and head_base,
// the head document's count before the tile, are then exact); otherwise
// their candidate and indexed bits go to the tile's mask slot (hmask) for the
// pass after the look-back.
// SIMPLE: no document starts or ends in [P0, P0 + kTileBytes] and the tile
// lies inside the input (every byte belongs to document hd, which starts at
// hs < P0), the escape state entering the tile is known, and defer is set.
// MIN: minify instead of index.  A byte is kept if it is not white space or
// lies inside a string (in the head region K marks the bytes whose fate flips
// with the incoming in-string state, F0 the kept bytes if it is 0), and the
// outputs are the kept bytes.
template <bool SIMPLE, bool MIN = false, int VAR = 0>
JSIDX_DEV void tile_local(const Args& a, uint32_t rows, Shared& sh, uint2* hmask, const uint32_t* first_row,
                          int64_t P0,
                          int64_t begin, int64_t end, int64_t d_first, int32_t hd, int64_t hs, uint32_t st_in,
                          bool defer, uint32_t head_base, TileFacts& T) {
  const uint32_t lane = prim::lane();
  uint32_t ce = st_in & 1u, cq = (st_in >> 1) & 1u, cp = (st_in >> 2) & 1u, cu = (st_in >> 3) & 1u;
  uint32_t cc = head_base;  // count of the open document before this row
  T.any_const = 0; T.lead_pos = kTileBytes; T.lead_reset = 0; T.qsens = 0;
  T.reset_any = 0; T.r0 = kTileBytes; T.elig0 = 0; T.head_rows = 0; T.a0 = 0; T.a1 = 0; T.tail_count = 0;
  T.tail_rows = 0;
  if (lane == 0) sh.he_valid = 0;

  // UTF-8 context entering the tile: the last bytes of the head document
  // before it (the word lies in the granule before P0, which holds document
  // bytes since hs < P0)
  U8Carry uc = u8_carry_zero();
  if (hs < P0 && begin < end) {
    uint32_t h = prim::load4(a.base + P0 - 4);
    const int64_t hlo = hs - (P0 - 4);  // bytes of the word before the document
    if (hlo > 0) h &= hlo >= 4 ? 0u : (~0u << (8 * hlo));
    uc = u8_carry_from_word(h);
  }

  uint32_t wn[8];
  if (first_row) {
#pragma unroll
    for (int k = 0; k < 8; k++) wn[k] = first_row[k];
  } else {
    load_segment<SIMPLE>(a, P0 + (int64_t)lane * kSegBytes, begin, end, wn);
  }
#if JSIDX_PREFETCH_ROWS > 1
  uint32_t wn2[8];
  if (rows > 1) load_segment<SIMPLE>(a, P0 + kRowBytes + (int64_t)lane * kSegBytes, begin, end, wn2);
#endif
  int32_t tab_cur = 0;  // first table entry not before the current row (table mode)
  const int32_t ntab = SIMPLE ? 0 : (int32_t)prim::readlane((uint32_t)sh.ntab, 0);
#pragma unroll 1
  for (int r = 0; r < (int)rows; r++) {
    const int32_t rel = r * kRowBytes + (int32_t)lane * kSegBytes;  // tile-relative
    const int64_t pos = P0 + rel;
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; k++) w[k] = wn[k];
#if JSIDX_PREFETCH_ROWS > 1
#pragma unroll
    for (int k = 0; k < 8; k++) wn[k] = wn2[k];
    if (r + 2 < (int)rows) load_segment<SIMPLE>(a, pos + 2 * kRowBytes, begin, end, wn2);  // two rows ahead
#else
    if (r + 1 < (int)rows) load_segment<SIMPLE>(a, pos + kRowBytes, begin, end, wn);  // prefetch
#endif

    // documents: starts in this segment (D), start right after it (d32),
    // document holding byte 0 (head), valid bytes (V)
    int32_t head = hd;
    uint32_t D = 0, d32 = 0, V = ~0u;
    if constexpr (!SIMPLE) {
      if (!sh.overflow) {
        // The table is sorted: a cursor moves past the starts before this
        // row, then the wave visits the row's own starts (usually none or
        // one), each lane taking the starts in or right after its segment
        // and the last start at or before its first byte (its document).
        const int32_t row0 = r * kRowBytes;
        while (tab_cur < ntab && (int32_t)prim::readlane((uint32_t)sh.tab[tab_cur], 0) < row0) tab_cur++;
        head = tab_cur - 1;
        for (int32_t i = tab_cur; i < ntab; i++) {
          const int32_t e = (int32_t)prim::readlane((uint32_t)sh.tab[i], 0);
          if (e > row0 + kRowBytes) break;
          const int32_t off = e - rel;
          if (off <= 0) head = i;
          if (off >= 0 && off < 32) D |= 1u << (uint32_t)off;
          if (off == 32) d32 = 1;
        }
      } else {
        head = doc_at(a, sh, P0, d_first, rel);
        for (int32_t i = head < 0 ? 0 : head;; i++) {
          if (d_first + i > (int64_t)a.ndocs) break;
          const int64_t o = doc_off(a, d_first + i);
          if (o < pos) continue;
          if (o > pos + 32) break;
          if (o == pos + 32) d32 = 1; else D |= 1u << (uint32_t)(o - pos);
        }
      }
      const int64_t vlo = begin - pos, vhi = end - pos;
      V = ge_mask((uint32_t)(vlo < 0 ? 0 : (vlo > 32 ? 32 : vlo))) &
          lt_mask((uint32_t)(vhi < 0 ? 0 : (vhi > 32 ? 32 : vhi)));
      if (head >= 0 && d_first + head >= (int64_t)a.ndocs) head = -1;
    }

    ClassMasks cm;
    if constexpr ((VAR & kVarNaiveClassify) != 0) {  // before w is dead
      SegWords sw;
#pragma unroll
      for (int k = 0; k < 8; k++) sw.w[k] = w[k];
      cm = classify_bytes(sw);
    }
    uint32_t pl[8];
    bit_planes(w, pl);
    if constexpr (!SIMPLE) {
      if (V != ~0u) {
#pragma unroll
        for (int k = 0; k < 8; k++) pl[k] &= V;
      }
    }
    if constexpr ((VAR & kVarNaiveClassify) != 0) {
      if constexpr (!SIMPLE) {
        cm.C &= V; cm.W &= V; cm.Q &= V; cm.B &= V;
      }
    } else {
      cm = classify_planes(pl);
    }

    // UTF-8: rows without non-ASCII bytes and with no sequence open from the
    // row before have no errors
    uint32_t errm = 0;
    if (prim::ballot(pl[7] != 0u) != 0ull || u8_carry_pending(uc)) {
      errm = utf8_errors(pl, D, SIMPLE ? 0u : ((D >> 1) | (d32 << 31)), &uc);
    } else {
      uc = u8_carry_zero();
    }

    // A plain row has no document start or end and only valid bytes: every
    // lane continues the document open at the row start.
    const bool plain = SIMPLE || prim::ballot(D != 0u || d32 != 0u || V != ~0u) == 0ull;

    // escapes: a segment with a non-backslash byte or a document start fixes
    // the escape state after it; an all-backslash segment (even length) keeps it
    if (!SIMPLE && !T.any_const) {
      // the tile's first byte that is not a backslash or starts a document
      // (used when the escape entering the tile is only known later)
      const uint64_t Kc = prim::ballot((cm.B != ~0u) || (D != 0u));
      if (Kc) {
        const int f = __builtin_ctzll(Kc);
        const uint32_t nbd = ~cm.B | D;
        const uint32_t pl0 = nbd ? (uint32_t)__builtin_ctz(nbd) : 0u;
        const uint32_t pf = prim::readlane(pl0, f);
        const uint32_t rf = prim::readlane((D >> pl0) & 1u, f);
        const uint32_t qf = prim::readlane((cm.Q >> pl0) & 1u, f);
        T.lead_pos = (uint32_t)(r * kRowBytes + f * kSegBytes) + pf;
        T.lead_reset = rf;
        T.qsens = rf ? 0u : qf;
        T.any_const = 1;
      }
    }
    uint32_t e_in = 0, OD = 0, EA = 0;
    bool done_e = false;
    if (plain) {
      if (prim::ballot(cm.B != 0u) == 0ull) {
        e_in = lane == 0 ? ce : 0u;
        OD = e_in;
        ce = 0u;
        done_e = true;
      } else if (prim::ballot(cm.B == ~0u) == 0ull) {
        const uint32_t eo = (uint32_t)__builtin_clz(~cm.B) & 1u;  // trailing run is odd
        e_in = shift_in1(eo << 31, &ce) & 1u;
        OD = odd_run_ends(cm.B & ~e_in) | e_in;
        done_e = true;
      }
    }
    if (!done_e) {
      const bool isconst = (cm.B != ~0u) || (D != 0u);
      const uint32_t hi_reset = D ? 31u - (uint32_t)__builtin_clz(D) : 0u;
      const uint32_t nb = ~(cm.B & ge_mask(hi_reset));
      const uint32_t eo = (nb ? (uint32_t)__builtin_clz(nb) : 32u) & 1u;
      const uint64_t Kc = prim::ballot(isconst);
      const uint64_t Ec = prim::ballot(eo != 0u);
      const uint64_t mk = Kc & lt_lanes();
      e_in = mk ? (uint32_t)((Ec >> msb64(mk)) & 1ull) : ce;
      if (Kc) ce = (uint32_t)((Ec >> msb64(Kc)) & 1ull);
      OD = escaped_bytes(cm.B, D, e_in, &EA);
    }
    const uint32_t Q = cm.Q & ~OD;

    // string ranges: prefix XOR, restarted at document starts
    const uint32_t PX = (VAR & kVarXorLoop) ? prefix_xor_loop(Q) : prefix_xor(Q);
    uint32_t R0 = PX;
    uint64_t Rs = 0;
    uint32_t uin = 0, first_reset = 32u, last_start = 0;
    if (plain) {
      const uint64_t Qb = prim::ballot((__builtin_popcount(Q) & 1u) != 0u);
      const uint32_t qin = (prim::mbcnt(Qb) & 1u) ^ cq;
      R0 ^= 0u - qin;
      cq ^= parity64(Qb);
      if (prim::ballot(errm != 0u)) cu = 1u;
    } else {
      uint32_t corr = 0, c_old = 0, rest = D;
      while (rest) {
        const uint32_t d = (uint32_t)__builtin_ctz(rest);
        rest &= rest - 1u;
        const uint32_t c_new = d ? ((PX >> (d - 1u)) & 1u) : 0u;
        if (c_new != c_old) corr ^= ge_mask(d);
        c_old = c_new;
      }
      R0 = PX ^ corr;
      last_start = D ? 31u - (uint32_t)__builtin_clz(D) : 0u;
      const uint32_t qv = D ? (R0 >> 31) : (uint32_t)(__builtin_popcount(Q) & 1);
      const uint32_t uv = (errm & ge_mask(last_start)) != 0u;
      Rs = prim::ballot(D != 0u);
      const uint64_t Qv = prim::ballot(qv != 0u);
      const uint64_t Uv = prim::ballot(uv != 0u);
      bool from_carry;
      const uint64_t sp = span_since_reset(Rs, &from_carry);
      uint32_t qin = parity64(Qv & sp);
      uin = (Uv & sp) ? 1u : 0u;
      if (from_carry) { qin ^= cq; uin |= cu; }
      first_reset = D ? (uint32_t)__builtin_ctz(D) : 32u;
      if (qin) R0 ^= lt_mask(first_reset);
      const uint64_t tl = tail_lanes(Rs);
      if (Rs) { cq = parity64(Qv & tl); cu = (Uv & tl) ? 1u : 0u; }
      else { cq ^= parity64(Qv); cu |= Uv ? 1u : 0u; }
    }

    // pseudo-structural candidates: the byte before is structural, white
    // space or a quote (or the byte starts a document)
    const uint32_t P0m = cm.C | cm.W | Q;
    const uint32_t PR = shift_in1(P0m, &cp) | D;

    if (r == 0 && !MIN) {
      const uint32_t other0 = (V & 1u) && !(D & 1u) && !((cm.C | cm.W | cm.Q) & 1u);
      T.elig0 = prim::readlane(other0, 0);
    }
    const uint32_t K = MIN ? (cm.W & V) : ((cm.C | Q | (PR & ~P0m)) & V);
    const uint32_t F0 = MIN ? ((~cm.W | R0) & V) : (K & ~(Q ^ R0));
    const bool had_reset = T.reset_any != 0;
    if (SIMPLE || (plain && defer && !had_reset)) {
      // the whole row lies in the head region
      prim::st_pair(hmask + r * kThreads + lane, K, F0);
      T.head_rows = (uint32_t)r + 1u;
      T.a0 += (uint32_t)__builtin_popcount(F0);
      T.a1 += (uint32_t)__builtin_popcount(F0 ^ K);
      continue;
    }
    if (plain) {
      // the whole row continues the open document; in the first pass its
      // positions are written after the tile has published its descriptor
      const int32_t h0 = prim::readlane((uint32_t)head, 0);
      const int64_t doff = doc_start(a, sh, P0, d_first, h0);
      if constexpr (MIN) {
        write_bytes(sh, reinterpret_cast<uint8_t*>(a.out_idx) + doff, (uint64_t)(end - doff), &cc, F0, w);
      } else if (defer) {
        sh.hF[r][lane] = F0;
        if (lane == 0) { sh.tr_doff[r] = doff; sh.tr_cc[r] = cc; }
        T.tail_rows |= 1u << r;
        cc += wave_sum((uint32_t)__builtin_popcount(F0));
      } else {
        write_row<(VAR & kVarDirectFlatten) == 0>(sh, a.out_idx + doff, (uint64_t)(end - doff), &cc, F0, (uint32_t)(pos - doff));
      }
      continue;
    }

    if (Rs && !had_reset) {
      const int fl = __builtin_ctzll(Rs);
      T.r0 = (uint32_t)(r * kRowBytes + fl * kSegBytes) + prim::readlane(first_reset, fl);
      T.reset_any = 1;
    }
    // head region of this lane: tile positions before the first document start
    const uint32_t hm = (uint32_t)rel >= T.r0 ? 0u : (T.r0 - (uint32_t)rel >= 32u ? ~0u : lt_mask(T.r0 - (uint32_t)rel));
    const bool row_has_head = !had_reset;
    if (defer && row_has_head) {
      prim::st_pair(hmask + r * kThreads + lane, K & hm, F0 & hm);
      T.head_rows = (uint32_t)r + 1u;
      T.a0 += (uint32_t)__builtin_popcount(F0 & hm);
      T.a1 += (uint32_t)__builtin_popcount((F0 ^ K) & hm);
    }

    // positions and per-document results of the pieces written now (none
    // while the whole row lies in a deferred head region)
    if (defer && !had_reset && Rs == 0ull && prim::ballot(d32 != 0u) == 0ull) continue;
    const uint32_t cv = (uint32_t)__builtin_popcount(F0 & ge_mask(last_start));
    const uint32_t cin = row_ranks(cv, Rs, &cc);
    const uint32_t wmask = defer ? ~hm : ~0u;
    uint32_t starts = D | 1u;
    while (starts) {
      const uint32_t st = (uint32_t)__builtin_ctz(starts);
      starts &= starts - 1u;
      const uint32_t nx = starts ? (uint32_t)__builtin_ctz(starts) : 32u;
      const bool ends_doc = nx < 32u || d32;
      const bool cont = (st == 0 && !(D & 1u));  // continues the previous lane's document
      const uint32_t segm = ge_mask(st) & lt_mask(nx);
      const uint32_t pu = ((errm & segm) != 0u ? 1u : 0u) | (cont ? uin : 0u);
      const bool deferred = defer && ((hm >> st) & 1u);
      if (deferred) {
        // the head document ends inside the head region: keep its flags
        if (ends_doc) {
          const uint32_t e = nx - 1u;
          sh.he_R0 = (R0 >> e) & 1u;
          sh.he_EA = (EA >> e) & 1u;
          sh.he_u = pu;
          sh.he_valid = 1;
        }
        continue;
      }
      const int32_t dloc = cont ? head : doc_at(a, sh, P0, d_first, rel + (int32_t)st);
      const int64_t dglob = d_first + dloc;
      if (dloc < 0 || dglob >= (int64_t)a.ndocs) continue;
      const int64_t doff = doc_start(a, sh, P0, d_first, dloc);
      uint32_t* out = a.out_idx + doff;
      const uint32_t rel_doc = (uint32_t)(pos - doff);
      const int64_t room = end - doff;
      const uint32_t lim = room > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)room;
      uint32_t f = F0 & wmask & segm;
      uint32_t kk = cont ? cin : 0u;
      if constexpr (MIN) {
        put_kept<0, false>(reinterpret_cast<uint8_t*>(a.out_idx) + doff, f, w, &kk, lim);
      } else {
        while (f) {
          const uint32_t j = (uint32_t)__builtin_ctz(f);
          f &= f - 1u;
          if (kk < lim) prim::st_out(out + kk, rel_doc + j);
          kk++;
        }
      }
      if (ends_doc) {
        const uint32_t e = nx - 1u;
        uint32_t err = 0;
        if (pu) err |= JSIDX_ERR_UTF8;
        if ((R0 >> e) & 1u) err |= JSIDX_ERR_UNCLOSED_STRING;
        if ((EA >> e) & 1u) err |= JSIDX_ERR_TRAILING_ESCAPE;
        if (kk == 0) err |= JSIDX_ERR_EMPTY;
        prim::st_out(a.out_n + dglob, kk);
        prim::st_out(a.out_err + dglob, err);
      }
    }
  }
  T.carry = ce | (cq << 1) | (cp << 2) | (cu << 3);
  T.tail_count = cc;
}

// ---- the look-back ----------------------------------------------------------
// Tiles are grouped in blocks of kBlockTiles.  A tile's incoming state comes
// from two windows, each read in one round trip: the blocks before its own
// (one block descriptor per lane, up to 64 blocks back; before block 0 lies
// the initial state) and the tiles of its own block before it (4 tile
// descriptors per lane).  The last tile of a block to publish its aggregate
// folds the block's tile descriptors into a block aggregate; the block's last
// tile publishes the block's inclusive value once it is resolved.  So no tile
// waits for a tile with a higher index, and the wait of a tile is bounded by
// the local passes of the tiles before it, not by a chain of look-backs.
//
// Lanes fold their descriptors (oldest first) into either a known state (if
// one is inclusive) or a transfer of the same kind as a tile's; the walk from
// the newest lane with a known state to the newest descriptor is then done
// for all lanes at once with ballots (segmented parity / OR scans) and one
// wave sum.
struct LaneFold {
  bool known, has, pending, blocked;
  uint32_t ks, kc;                       // known state and count
  uint32_t fr, fec, fev, fp, fq, fu;     // transfer: reset, e const?, e value, p, q, u
  uint32_t C0, C1, E0;                   // counts for q_in = 0 / 1; first tile's elig0
  uint32_t b0, b1;                       // an escape-sensitive tile sees e = 1
                                         //   if the run starts with e_in = 0 / 1
};

JSIDX_DEV LaneFold fold_empty() {
  LaneFold L;
  L.known = L.has = L.pending = L.blocked = false;
  L.ks = L.kc = 0; L.fr = L.fec = L.fev = L.fp = L.fq = L.fu = 0; L.C0 = L.C1 = L.E0 = 0; L.b0 = L.b1 = 0;
  return L;
}

JSIDX_DEV LaneFold fold_known(uint32_t state, uint32_t count) {
  LaneFold L = fold_empty();
  L.known = true; L.ks = state; L.kc = count;
  return L;
}

JSIDX_DEV void fold_desc(LaneFold& L, uint64_t d, bool valid) {
  if (!valid) return;
  const uint32_t fl = d_flag(d);
  if (fl == kNone) { L.pending = true; return; }
  if (fl == kInc) {
    L.known = true; L.has = false; L.pending = false; L.blocked = false;
    L.ks = d_state(d); L.kc = d_count(d);
    return;
  }
  const uint32_t T = d_table(d), c0 = d_c0(d), c1 = d_c1(d), el = d_elig0(d), es = d_esens(d);
  const uint32_t ent0 = (T >> 2) & 7u, ent1 = (T >> 5) & 7u;
  const uint32_t Bec = ((ent0 ^ ent1) & 1u) == 0u;  // e_out does not depend on e_in
  const uint32_t Bev = ent0 & 1u, Bq = (ent0 >> 1) & 1u, Bp = (ent0 >> 2) & 1u, Bu = (T >> 1) & 1u;
  const uint32_t Br = T & 1u;
  if (L.known) {
    if (es && (L.ks & 1u)) L.blocked = true;
    const uint32_t q = (L.ks >> 1) & 1u, p = (L.ks >> 2) & 1u;
    L.kc = Br ? c0 : L.kc + (q ? c1 : c0 + (p & el));
    L.ks = tab_apply(T, L.ks);
    return;
  }
  if (!L.has) {
    L.has = true;
    L.fr = Br; L.fec = Bec; L.fev = Bev; L.fp = Bp; L.fq = Bq; L.fu = Bu;
    L.C0 = c0; L.C1 = Br ? c0 : c1; L.E0 = Br ? 0u : el;
    L.b0 = 0; L.b1 = es;
    return;
  }
  L.b0 |= es & (L.fec ? L.fev : 0u);
  L.b1 |= es & (L.fec ? L.fev : 1u);
  if (Bec) { L.fec = 1; L.fev = Bev; }
  if (Br) {
    L.fr = 1; L.fq = Bq; L.fu = Bu; L.C0 = L.C1 = c0;
  } else {
    const uint32_t qa0 = L.fq;                       // q entering B when the run starts with q = 0
    const uint32_t qa1 = L.fr ? L.fq : (1u ^ L.fq);  // ... with q = 1
    L.C0 += qa0 ? c1 : c0 + (L.fp & el);
    L.C1 += qa1 ? c1 : c0 + (L.fp & el);
    L.fq ^= Bq;
    L.fu |= Bu;
  }
  L.fp = Bp;
}

// A := A then B (B covers the newer descriptors).
JSIDX_DEV void compose(LaneFold& A, const LaneFold& B) {
  if (B.known) { A = B; return; }
  if (!B.has) return;
  if (A.known) {
    const uint32_t e_in = A.ks & 1u, q_in = (A.ks >> 1) & 1u, p_in = (A.ks >> 2) & 1u, u_in = (A.ks >> 3) & 1u;
    if (e_in ? B.b1 : B.b0) A.blocked = true;
    const uint32_t e = B.fec ? B.fev : e_in;
    const uint32_t q = B.fr ? B.fq : (q_in ^ B.fq);
    const uint32_t u = B.fr ? B.fu : (u_in | B.fu);
    A.kc = B.fr ? B.C0 : A.kc + (q_in ? B.C1 : B.C0 + (p_in & B.E0));
    A.ks = e | (q << 1) | (B.fp << 2) | (u << 3);
    return;
  }
  if (!A.has) { A = B; return; }
  const uint32_t ea0 = A.fec ? A.fev : 0u, ea1 = A.fec ? A.fev : 1u;  // e entering B
  A.b0 |= ea0 ? B.b1 : B.b0;
  A.b1 |= ea1 ? B.b1 : B.b0;
  if (B.fec) { A.fec = 1; A.fev = B.fev; }
  if (B.fr) {
    A.fr = 1; A.fq = B.fq; A.fu = B.fu; A.C0 = A.C1 = B.C0;
  } else {
    const uint32_t qa0 = A.fq, qa1 = A.fr ? A.fq : (1u ^ A.fq);
    const uint32_t pe = A.fp & B.E0;
    A.C0 += qa0 ? B.C1 : B.C0 + pe;
    A.C1 += qa1 ? B.C1 : B.C0 + pe;
    A.fq ^= B.fq;
    A.fu |= B.fu;
  }
  A.fp = B.fp;
}

// Transfer flags of a fold in one word (for lane shuffles); the counts travel
// separately (C0 holds the known count of a known fold).
JSIDX_DEV uint32_t fold_flags(const LaneFold& L) {
  return (L.known ? 1u : 0u) | (L.has ? 2u : 0u) | (L.blocked ? 4u : 0u) | (L.fr << 3) | (L.fec << 4) |
         (L.fev << 5) | (L.fp << 6) | (L.fq << 7) | (L.fu << 8) | (L.E0 << 9) | (L.b0 << 10) | (L.b1 << 11) |
         (L.ks << 12);
}
JSIDX_DEV LaneFold fold_unpack(uint32_t f, uint32_t c0, uint32_t c1) {
  LaneFold L = fold_empty();
  L.known = f & 1u; L.has = (f >> 1) & 1u; L.blocked = (f >> 2) & 1u;
  L.fr = (f >> 3) & 1u; L.fec = (f >> 4) & 1u; L.fev = (f >> 5) & 1u; L.fp = (f >> 6) & 1u;
  L.fq = (f >> 7) & 1u; L.fu = (f >> 8) & 1u; L.E0 = (f >> 9) & 1u; L.b0 = (f >> 10) & 1u; L.b1 = (f >> 11) & 1u;
  L.ks = (f >> 12) & 0xFu;
  L.kc = c0; L.C0 = c0; L.C1 = c1;
  return L;
}

// ---- block descriptors: 3 words per block ----------------------------------
// [0] aggregate: bits 0..1 kAgg, 2..10 transfer flags (fr fec fev fp fq fu E0
//     b0 b1), 11..34 C0, 35..58 C1, 59..63 low epoch bits;
// [1] inclusive and [2] incoming (state and count before the block), both in
//     the tile inclusive format.
// All block words are cleared at the end of every launch.
constexpr uint64_t kAggEpochMask = 31;
JSIDX_DEV uint64_t* block_desc(const Args& a) { return a.ws->desc + a.cap_tiles; }
// Head-region masks: one slot of rows * kThreads pairs per tile, row after
// row (a tile writes and later reads back one contiguous slot, which stays
// in the caches between the two).
JSIDX_DEV uint2* head_masks(const Args& a, int64_t t, uint32_t rows) {
  return reinterpret_cast<uint2*>(reinterpret_cast<uint8_t*>(a.ws) + mask_offset(a.cap_tiles)) +
         t * ((int64_t)rows * kThreads);
}
JSIDX_DEV uint32_t* block_count(const Args& a) {
  return reinterpret_cast<uint32_t*>(block_desc(a) + 3 * blocks_for_tiles(a.cap_tiles));
}

JSIDX_DEV LaneFold read_block(const Args& a, int64_t bb, uint32_t epoch) {
  if (bb < -1) return fold_empty();
  if (bb == -1) return fold_known(0u, 0u);  // the state before the input
  const uint64_t* bd = block_desc(a) + 3 * bb;
  const uint64_t inc = prim::ld_agent(bd + 1);
  if (d_current(inc, epoch) && d_flag(inc) == kInc) return fold_known(d_state(inc), d_count(inc));
  const uint64_t w = prim::ld_agent(bd);
  LaneFold L = fold_empty();
  if (d_flag(w) != kAgg || (w >> 59) != ((uint64_t)epoch & kAggEpochMask)) {
    L.pending = true;
    return L;
  }
  const uint32_t f = (uint32_t)(w >> 2) & 0x1FFu;
  L.has = true;
  L.fr = f & 1u; L.fec = (f >> 1) & 1u; L.fev = (f >> 2) & 1u; L.fp = (f >> 3) & 1u; L.fq = (f >> 4) & 1u;
  L.fu = (f >> 5) & 1u; L.E0 = (f >> 6) & 1u; L.b0 = (f >> 7) & 1u; L.b1 = (f >> 8) & 1u;
  L.C0 = (uint32_t)(w >> 11) & 0xFFFFFFu;
  L.C1 = (uint32_t)(w >> 35) & 0xFFFFFFu;
  return L;
}

struct WalkOut {
  bool ready, blocked;
  uint32_t state, count;
};

// From the newest lane with a known state to the end of lane 0's run (lane 0
// holds the newest descriptors): the state and the count of the open document.
JSIDX_DEV WalkOut walk(const LaneFold& L) {
  const uint32_t lane = prim::lane();
  WalkOut w;
  w.ready = false; w.blocked = false; w.state = 0; w.count = 0;
  const uint64_t Kn = prim::ballot(L.known);
  const int k = Kn ? __builtin_ctzll(Kn) : 64;
  const uint64_t below = lanes_below(k);
  const uint64_t pend = prim::ballot(L.pending) & (below | (k < 64 ? (1ull << k) : 0ull));
  if (Kn == 0 || pend) return w;
  // known start: lane k, after its newest descriptor
  const uint32_t ks = prim::readlane(L.ks, k), kc = prim::readlane(L.kc, k);
  const uint32_t kblk = prim::readlane(L.blocked ? 1u : 0u, k);
  // lanes below k are transfers; lane 0 is the newest
  const uint64_t Ec = prim::ballot(L.has && L.fec) & below;
  const uint64_t Ev = prim::ballot(L.fev != 0u);
  const uint64_t Rs = prim::ballot(L.has && L.fr) & below;
  const uint64_t Qv = prim::ballot(L.fq != 0u);
  const uint64_t Uv = prim::ballot(L.fu != 0u);
  const uint64_t above = ~lanes_below((int)lane + 1);  // older lanes
  // escape at this lane's entry: nearest older lane that fixes it, else ks
  const uint64_t me = Ec & above;
  const uint32_t e_ent = me ? (uint32_t)((Ev >> __builtin_ctzll(me)) & 1ull) : (ks & 1u);
  // in-string and UTF-8 state at entry: from the nearest older reset lane
  const uint64_t mr = Rs & above;
  const uint64_t span = (mr ? lanes_below(__builtin_ctzll(mr) + 1) : below) & above;
  uint32_t q_ent = parity64(Qv & span);
  uint32_t u_ent = (Uv & span) ? 1u : 0u;
  if (!mr) { q_ent ^= (ks >> 1) & 1u; u_ent |= (ks >> 3) & 1u; }
  uint32_t p_ent = prim::shfl(L.fp, (int)((lane + 1u) & 63u));
  if ((int)lane + 1 >= k) p_ent = (ks >> 2) & 1u;
  const bool blk = L.has && (e_ent ? L.b1 : L.b0);
  w.blocked = (prim::ballot(blk) & below) != 0ull || (kblk != 0u);
  // count: from the newest reset lane below k (absolute), else from kc
  uint32_t contrib = 0;
  if (L.has) contrib = L.fr ? L.C0 : (q_ent ? L.C1 : L.C0 + (p_ent & L.E0));
  const int rn = Rs ? __builtin_ctzll(Rs) : -1;
  const uint64_t cm = rn >= 0 ? lanes_below(rn + 1) : below;
  const uint32_t sum = wave_sum(((cm >> lane) & 1ull) ? contrib : 0u);
  // state after lane 0
  if (k == 0) {
    w.state = ks;
  } else {
    const uint32_t e_after = L.fec ? L.fev : e_ent;
    const uint32_t q_after = L.fr ? L.fq : (q_ent ^ L.fq);
    const uint32_t u_after = L.fr ? L.fu : (u_ent | L.fu);
    w.state = prim::readlane(e_after | (q_after << 1) | (L.fp << 2) | (u_after << 3), 0);
  }
  w.count = rn >= 0 ? sum : kc + sum;
  w.ready = true;
  return w;
}

// Back-off between polls: 1, 2, 4, then 16 sleeps of 64 clocks.
JSIDX_DEV void poll_sleep(uint32_t polls) {
  const int n = polls < 2 ? 1 : (polls < 4 ? 2 : (polls < 8 ? 4 : 16));
  for (int i = 0; i < n; i++) prim::sleep();
}

// The last tile of block b to publish its descriptor folds the block (each
// lane folds 4 tile descriptors, then lanes combine pairwise, the older
// partner at lane + s) and publishes the block aggregate.  Unless the fold is
// already an inclusive value, it then walks the blocks before (one per lane,
// up to 64 back) for the state entering block b and publishes the block's
// inclusive value, which the tiles of block b + 1 wait for.
JSIDX_DEV void compose_block(const Args& a, int64_t b, int64_t ntiles, uint32_t epoch) {
  const uint32_t lane = prim::lane();
  const int64_t lo = b * kBlockTiles;
  const int64_t hi = lo + kBlockTiles < ntiles ? lo + kBlockTiles : ntiles;
  const int64_t j0 = hi - 1 - 4 * (int64_t)lane;
  uint64_t* bd = block_desc(a) + 3 * b;
  LaneFold L;
  for (uint32_t polls = 0;; polls++) {
    L = fold_empty();
    uint64_t d[4];
#pragma unroll
    for (int m = 0; m < 4; m++) d[m] = (j0 - m >= lo) ? ld_desc(a.ws, j0 - m) : 0ull;
#pragma unroll
    for (int m = 3; m >= 0; m--) {
      const bool valid = j0 - m >= lo;
      fold_desc(L, (valid && d_current(d[m], epoch)) ? d[m] : 0ull, valid);
    }
    // every tile of the block has published (the counter says so); a stale
    // read is retried
    if (prim::ballot(L.pending && !L.known) == 0ull) break;
    if (polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); return; }
    poll_sleep(polls);
  }
#pragma unroll 1
  for (int s = 1; s < 64; s <<= 1) {
    const uint32_t f = fold_flags(L), c0 = L.known ? L.kc : L.C0, c1 = L.C1;
    const int src = (int)(lane + (uint32_t)s) & 63;
    const uint32_t of = prim::shfl(f, src), oc0 = prim::shfl(c0, src), oc1 = prim::shfl(c1, src);
    if ((lane & (uint32_t)(2 * s - 1)) == 0u) {
      LaneFold O = fold_unpack(of, oc0, oc1);
      compose(O, L);
      L = O;
    }
  }
  // lane 0 holds the block's fold
  const uint32_t bf = prim::readlane(fold_flags(L), 0);
  const uint32_t b0 = prim::readlane(L.known ? L.kc : L.C0, 0), b1 = prim::readlane(L.C1, 0);
  const LaneFold B = fold_unpack(bf, b0, b1);
  if (lane == 0) {
    if (B.known && !B.blocked) {
      prim::st_agent(bd + 1, make_inc(B.ks, 0u, B.kc, epoch));
    } else if (B.has) {
      const uint32_t tf = B.fr | (B.fec << 1) | (B.fev << 2) | (B.fp << 3) | (B.fq << 4) | (B.fu << 5) |
                          (B.E0 << 6) | (B.b0 << 7) | (B.b1 << 8);
      prim::st_agent(bd, (uint64_t)kAgg | ((uint64_t)tf << 2) | ((uint64_t)(B.C0 & 0xFFFFFFu) << 11) |
                             ((uint64_t)(B.C1 & 0xFFFFFFu) << 35) | (((uint64_t)epoch & kAggEpochMask) << 59));
    }
    // a known but blocked fold publishes nothing here: the block's inclusive
    // value follows from its last tile once the escape-sensitive tile has
    // redone its pass
  }
  if (B.known || !B.has) return;
  // the state entering block b (walk over the blocks before), then the
  // block's inclusive value
  uint32_t es = 0, ec = 0;
  if (b > 0) {
    for (uint32_t polls = 0;; polls++) {
      const WalkOut w2 = walk(read_block(a, b - 1 - (int64_t)lane, epoch));
      if (w2.ready && !w2.blocked) { es = w2.state; ec = w2.count; break; }
      if (polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); return; }
      poll_sleep(polls);
    }
  }
  if (lane == 0) {
    LaneFold K = fold_known(es, ec);
    compose(K, B);
    if (!K.blocked) prim::st_agent(bd + 1, make_inc(K.ks, 0u, K.kc, epoch));
  }
}

// State entering tile t and the count of its head document before it.
JSIDX_DEV void look_back(const Args& a, int64_t t, uint32_t epoch, uint32_t* s_out, uint32_t* base_out) {
  const uint32_t lane = prim::lane();
  Workspace* ws = a.ws;
  const int64_t b = t / kBlockTiles, lo = b * kBlockTiles;
  bool have_blk = b == 0;
  uint32_t bs = 0, bc = 0;  // state and count entering the block (block 0: the initial state)
  for (uint32_t polls = 0;; polls++) {
    if (polls > prim::kSpinLimit) {  // never expected: give up, flag it
      prim::st_agent32(&ws->diag, 1u);
      *s_out = 0; *base_out = 0;
      return;
    }
    if (!have_blk) {
      // the previous block's inclusive value (not needed if this block's
      // tiles before t hold an inclusive descriptor)
      uint64_t v = 0;
      if (lane == 0) v = prim::ld_agent(block_desc(a) + 3 * (b - 1) + 1);
      const uint32_t lo32 = prim::readlane((uint32_t)v, 0), hi32 = prim::readlane((uint32_t)(v >> 32), 0);
      v = ((uint64_t)hi32 << 32) | lo32;
      if (d_current(v, epoch) && d_flag(v) == kInc) { have_blk = true; bs = d_state(v); bc = d_count(v); }
    }
    // the tiles of this block before t; the tile before the block holds the
    // block's incoming value
    const int64_t j0 = t - 1 - 4 * (int64_t)lane;  // this lane's newest tile
    uint64_t d[4];
#pragma unroll
    for (int m = 0; m < 4; m++) {
      const int64_t j = j0 - m;
      d[m] = j >= lo ? ld_desc(ws, j) : ((j == lo - 1 && have_blk) ? make_inc(bs, 0u, bc, epoch) : 0ull);
    }
    // Ready when some lane holds an inclusive descriptor and every descriptor
    // newer than the newest one is published: only then fold (a failed poll
    // costs a few operations).
    {
      uint32_t m_inc = 4, m_none = 4;  // newest inclusive / unpublished in this lane
#pragma unroll
      for (int m = 3; m >= 0; m--) {
        if (j0 - m < lo - 1) continue;
        const uint32_t fl = d_current(d[m], epoch) ? d_flag(d[m]) : (uint32_t)kNone;
        if (fl == kInc) m_inc = (uint32_t)m;
        if (fl == kNone) m_none = (uint32_t)m;
      }
      const uint64_t Ki = prim::ballot(m_inc < 4u);
      const int ki = Ki ? __builtin_ctzll(Ki) : 64;
      const uint64_t Pn = prim::ballot(m_none < m_inc) & (lanes_below(ki) | (ki < 64 ? (1ull << ki) : 0ull));
      if (Ki == 0ull || Pn != 0ull) {
        prim::trace_count(t, 8);
        poll_sleep(polls);
        continue;
      }
    }
    LaneFold L = fold_empty();
#pragma unroll
    for (int m = 3; m >= 0; m--) {
      const bool valid = j0 - m >= lo - 1;
      fold_desc(L, (valid && d_current(d[m], epoch)) ? d[m] : 0ull, valid);
    }
    prim::trace_count(t, 8);
    const WalkOut w = walk(L);
    if (!w.ready || w.blocked) {
      // some tile's counts depend on an escape that turned out to be set; that
      // tile redoes its local pass and publishes an exact inclusive value
      prim::trace_count(t, 10);
      poll_sleep(polls);
      continue;
    }
    *s_out = w.state;
    *base_out = w.count;
    return;
  }
}

// ---------------------------------------------------------------------------
// Per-tile set-up: the documents of the tile (LDS table) and the escape state
// entering it.
struct TileSetup {
  int64_t t, P0, d_first, hs;
  uint32_t rows;  // rows of the launch's tiles
  int32_t hd;
  bool hd_ok, simple;
  uint32_t e_T, e_known;
  uint32_t w0[8];  // this lane's segment of row 0, loaded first
};

JSIDX_DEV TileSetup begin_tile(const Args& a, uint32_t rows, Shared& sh, int64_t t, int64_t pos_g0, int64_t begin,
                               int64_t end, int64_t ntiles) {
  const uint32_t lane = prim::lane();
  TileSetup S;
  S.rows = rows;
  S.t = t;
  const int64_t tb = (int64_t)rows * kRowBytes;
  S.P0 = pos_g0 + t * tb;  // position of tile byte 0
  const int64_t P0 = S.P0, Pend = P0 + tb;
  // the first row's loads go out before anything else of the tile
  load_segment<false>(a, P0 + (int64_t)lane * kSegBytes, begin, end, S.w0);
  // d_first: the first document whose end is at or after the tile start.
  int64_t d_first;
  {
    int64_t lo = 0, hi = (int64_t)a.ndocs - 1;
    while (lo < hi) {
      const int64_t step = (hi - lo + 64) / 64;
      const int64_t d = lo + (int64_t)lane * step;
      const bool pr = d <= hi && doc_off(a, d + 1) >= P0;
      const uint64_t b = prim::ballot(pr);
      const int64_t f = b ? (int64_t)__builtin_ctzll(b) : -1;
      int64_t nprobe = (hi - lo) / step;  // last valid probe lane
      if (nprobe > 63) nprobe = 63;
      const int64_t nlo = f > 0 ? lo + (f - 1) * step + 1 : (f == 0 ? lo : lo + nprobe * step + 1);
      hi = f >= 0 ? lo + f * step : hi;
      lo = nlo;
    }
    d_first = lo;
  }
  S.d_first = d_first;
  // Table of starts of documents d_first.. up to Pend, relative to P0
  // (entry 0 clamped at -1).  Empty documents owned by this tile are
  // finished here: the tile owning a position owns the empty documents there.
  {
    int32_t count = 0;
    for (int64_t i0 = 0;; i0 += kThreads) {
      const int64_t d = d_first + i0 + lane;
      bool in = d <= (int64_t)a.ndocs;
      const int64_t o = in ? doc_off(a, d) : 0;
      in = in && o <= Pend;
      if (in && i0 + lane < kDocCap + 1) {
        const int64_t r = o - P0;
        sh.tab[i0 + lane] = (int32_t)(r < -1 ? -1 : r);
      }
      if (in && d < (int64_t)a.ndocs) {
        const int64_t o2 = doc_off(a, d + 1);
        const bool owned = (o >= P0 && o < Pend) || (o == end && t == ntiles - 1);
        if (o2 == o && owned) {
          prim::st_out(a.out_n + d, 0u);
          prim::st_out(a.out_err + d, JSIDX_ERR_EMPTY);
        }
      }
      const int n_in = __builtin_popcountll(prim::ballot(in));
      count += n_in;
      if (n_in < kThreads) break;
    }
    if (lane == 0) {
      sh.d_first = d_first;
      sh.first_off = doc_off(a, d_first);
      sh.ntab = count;
      sh.overflow = count > kDocCap + 1;
    }
  }
  prim::wave_sync();
  prim::trace(t, 1);

  // ---- escape state entering the tile -------------------------------------
  // Only the backslash run ending right before the tile decides it (odd run:
  // the tile's first byte is escaped), so it is read from the bytes before the
  // tile instead of waiting for the look-back.  Usually the byte before is
  // not a backslash; otherwise the wave measures the run, 1 KiB per step.
  // Runs longer than kEscSteps KiB leave it to the look-back.
  S.hd = doc_at(a, sh, P0, d_first, 0);
  S.hd_ok = S.hd >= 0 && d_first + S.hd < (int64_t)a.ndocs;
  S.hs = S.hd_ok ? doc_start(a, sh, P0, d_first, S.hd) : P0;  // head document start
  const int64_t hs = S.hs;
  S.e_T = 0; S.e_known = 1;
  if (t > 0 && hs < P0) {
    const uint32_t w0 = prim::load4(a.base + P0 - 4);  // granule [P0-16, P0) holds document bytes
    if ((w0 >> 24) == 0x5Cu) {
      S.e_known = 0;
      for (int step = 0; step < kEscSteps; step++) {
        const int64_t c = P0 - (int64_t)kThreads * 16 * step - 16 * ((int64_t)lane + 1);  // lane 0 nearest
        uint32_t bs = 0;  // bit i: byte c+i is a backslash of the document
        if (c + 16 > hs) {
          const uint4 v = prim::load16(a.base + c);
          const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const uint32_t x = wv[k] ^ 0x5C5C5C5Cu;  // zero bytes are backslashes
            const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
            bs |= ((z >> 7) & 1u) << (4 * k) | ((z >> 15) & 1u) << (4 * k + 1) |
                  ((z >> 23) & 1u) << (4 * k + 2) | ((z >> 31) & 1u) << (4 * k + 3);
          }
          if (c < hs) bs &= ~0u << (uint32_t)(hs - c);
        }
        const uint32_t trail = (uint32_t)__builtin_clz(~(bs << 16));  // run at the top, 0..16
        const uint64_t full = prim::ballot(trail >= 16u);
        const uint64_t notfull = ~full;
        if (notfull) {
          const int f = __builtin_ctzll(notfull);
          const uint32_t run = (uint32_t)f * 16u + prim::readlane(trail, f);
          S.e_T = run & 1u;  // runs of whole steps are even
          S.e_known = 1;
          break;
        }
      }
    }
  }
  S.simple = !sh.overflow && sh.ntab == 1 && sh.tab[0] < 0 && S.hd_ok && S.e_known;
  prim::trace(t, 5);
  return S;
}

// What a tile still owes after publishing: its look-back, its inclusive value
// (unless already published) and its head region (wave-uniform).
struct Pending {
  bool valid;
  TileSetup S;
  uint32_t table, cnt0, cnt1, esens, elig0, reset_any, r0, head_rows, carry, tail_count;
  bool inc_done;
  uint32_t he_valid, he_R0, he_EA, he_u;
};

// The local pass of a tile, its descriptor, its block's fold if it is the
// block's last to publish, and the positions that need nothing from earlier
// tiles.  The head region's masks go to the tile's slot in the workspace.
template <bool MIN, int VAR = 0>
JSIDX_DEV Pending start_tile(const Args& a, Shared& sh, const TileSetup& S, int64_t begin, int64_t end,
                             int64_t ntiles, uint32_t epoch) {
  const uint32_t lane = prim::lane();
  Workspace* ws = a.ws;
  const int64_t t = S.t, P0 = S.P0;
  uint2* hmask = head_masks(a, t, S.rows);
  TileFacts T;
  if (S.simple)
    tile_local<true, MIN, VAR>(a, S.rows, sh, hmask, S.w0, P0, begin, end, S.d_first, S.hd, S.hs, S.e_T, true, 0u, T);
  else
    tile_local<false, MIN, VAR>(a, S.rows, sh, hmask, S.w0, P0, begin, end, S.d_first, S.hd, S.hs, S.e_T, true, 0u, T);
  prim::trace(t, 2);
  Pending R;
  R.valid = true;
  R.S = S;
  {
    const uint32_t q0 = (T.carry >> 1) & 1u, p0 = (T.carry >> 2) & 1u, u0 = (T.carry >> 3) & 1u;
    const uint32_t e_last = T.carry & 1u;
    uint32_t table = T.reset_any | (u0 << 1);
#pragma unroll
    for (uint32_t e = 0; e < 2; e++) {
      // with the incoming escape known, both entries are the tile's outcome
      const uint32_t eo = (T.any_const || S.e_known) ? e_last : e;
      const uint32_t flip = S.e_known ? 0u : (e & T.qsens);
      const uint32_t qo = T.reset_any ? q0 : (q0 ^ flip);
      const uint32_t po = p0 ^ (flip & (T.lead_pos == S.rows * (uint32_t)kRowBytes - 1u ? 1u : 0u));
      table |= (eo | (qo << 1) | (po << 2)) << (2 + 3 * e);
    }
    R.table = table;
    if (T.reset_any) {
      R.cnt0 = R.cnt1 = T.tail_count;
    } else {
      R.cnt0 = wave_sum(T.a0);
      R.cnt1 = wave_sum(T.a1);
    }
  }
  R.esens = S.e_known ? 0u : (T.qsens | ((T.lead_reset && T.lead_pos > 0) ? 1u : 0u));
  R.elig0 = T.elig0; R.reset_any = T.reset_any; R.r0 = T.r0; R.head_rows = T.head_rows;
  R.carry = T.carry; R.tail_count = T.tail_count;
  // Publish.  After a document start nothing depends on earlier tiles, so a
  // tile holding one publishes its inclusive value right away.
  R.inc_done = T.reset_any != 0;
  if (lane == 0) {
    if (R.inc_done) {
      const uint64_t inc = make_inc(T.carry, 1u, T.tail_count, epoch);
      st_desc(ws, t, inc);
      if (t % kBlockTiles == kBlockTiles - 1) prim::st_agent(block_desc(a) + 3 * (t / kBlockTiles) + 1, inc);
    } else {
      st_desc(ws, t, make_agg(R.table, R.cnt0, R.cnt1, T.elig0, R.esens, epoch));
    }
  }
  {
    // count the block's published tiles; the last one folds the block
    const int64_t blk = t / kBlockTiles;
    const int64_t nblk = (ntiles - blk * kBlockTiles) < kBlockTiles ? (ntiles - blk * kBlockTiles) : kBlockTiles;
    prim::wait_mem();  // the descriptor is written before it is counted
    uint32_t old = 0;
    if (lane == 0) old = prim::add_agent32(block_count(a) + blk, 1u);
    old = prim::readlane(old, 0);
    if ((int64_t)old == nblk - 1) {
      compose_block(a, blk, ntiles, epoch);
      if (lane == 0) prim::st_agent32(block_count(a) + blk, 0u);  // ready for the next launch
    }
  }
  prim::wave_sync();
  // the head document's flags, if it ends inside the head region
  R.he_valid = sh.he_valid; R.he_R0 = sh.he_R0; R.he_EA = sh.he_EA; R.he_u = sh.he_u;
  // plain rows after a document start
  uint32_t rows = T.tail_rows;
  while (rows) {
    const int r = __builtin_ctz(rows);
    rows &= rows - 1u;
    const int64_t doff = sh.tr_doff[r];
    uint32_t cc = sh.tr_cc[r];
    const int64_t pos = P0 + (int64_t)r * kRowBytes + (int64_t)lane * kSegBytes;
    write_row<(VAR & kVarDirectFlatten) == 0>(sh, a.out_idx + doff, (uint64_t)(end - doff), &cc, sh.hF[r][lane],
                                              (uint32_t)(pos - doff));
  }
  prim::wave_sync();
  return R;
}

// The look-back of a published tile, the rare exact second pass (when the
// escape carried in turns out to change the tile's head), its inclusive
// value, and its head region's positions and head document's result.
template <bool MIN, int VAR = 0>
JSIDX_DEV void finish_tile(const Args& a, Shared& sh, const Pending& R, int64_t pos_g0, int64_t begin, int64_t end,
                           int64_t ntiles, uint32_t epoch) {
  const uint32_t lane = prim::lane();
  Workspace* ws = a.ws;
  const TileSetup& S = R.S;
  const int64_t t = S.t, P0 = S.P0;
  const bool hvalid = S.hd_ok && R.r0 > 0;
  if (R.inc_done && !hvalid) {  // no head region: nothing needs the look-back
    prim::trace(t, 3);
    prim::trace(t, 4);
    prim::trace(t, 7);
    return;
  }
  uint32_t s_in = 0, base = 0;
  look_back(a, t, epoch, &s_in, &base);
  prim::trace(t, 3);
  if ((s_in & 1u) && R.esens) {
    // exact second pass with the incoming state now known; it writes every
    // position of the tile itself
    prim::trace_count(t, 9);
    const TileSetup S2 = begin_tile(a, S.rows, sh, t, pos_g0, begin, end, ntiles);
    TileFacts T;
    tile_local<false, MIN, VAR>(a, S.rows, sh, head_masks(a, t, S.rows), S2.w0, P0, begin, end, S2.d_first, S2.hd, S2.hs, s_in, false, base,
                      T);
    if (lane == 0 && !R.inc_done) {
      const uint64_t inc = make_inc(T.carry, T.reset_any, T.tail_count, epoch);
      st_desc(ws, t, inc);
      if (t % kBlockTiles == kBlockTiles - 1) prim::st_agent(block_desc(a) + 3 * (t / kBlockTiles) + 1, inc);
    }
    prim::wave_sync();
    prim::trace(t, 4);
    prim::trace(t, 7);
    return;
  }
  if (lane == 0 && !R.inc_done) {
    const uint32_t q = (s_in >> 1) & 1u, p = (s_in >> 2) & 1u;
    const uint32_t cnt = R.reset_any ? R.cnt0 : base + (q ? R.cnt1 : R.cnt0 + (p & R.elig0));
    const uint64_t inc = make_inc(tab_apply(R.table, s_in), R.reset_any, cnt, epoch);
    st_desc(ws, t, inc);
    if (t % kBlockTiles == kBlockTiles - 1) prim::st_agent(block_desc(a) + 3 * (t / kBlockTiles) + 1, inc);
  }
  prim::trace(t, 4);

  // ---- head region: positions and the head document's result ---------------
  if (hvalid) {
    const uint32_t qT = (s_in >> 1) & 1u;
    const uint32_t pfix = (((s_in >> 2) & 1u) && R.elig0 && !qT) ? 1u : 0u;
    const uint32_t uT = (s_in >> 3) & 1u;
    uint32_t* out = a.out_idx + S.hs;
    // ranks of the head document stay below end - hs unless a look-back
    // wait gave up; rows that could pass it check every write
    const uint64_t lim = (uint64_t)(end - S.hs);
    const uint32_t rel0 = (uint32_t)(P0 - S.hs) + lane * (uint32_t)kSegBytes;
    // All rows' masks are loaded at once (one round trip); their indexed bits
    // go to the wave's LDS rows (free now: the tail rows of the tile started
    // since were written right after it published), so that the writes below
    // never wait on a load.
    const uint2* hmask = head_masks(a, t, S.rows);
    uint32_t Fr[kRows];
#pragma unroll
    for (int r = 0; r < kRows; r++) {
      uint2 kf;
      kf.x = 0u; kf.y = 0u;
      if ((uint32_t)r < R.head_rows) kf = prim::ld_pair(hmask + r * kThreads + lane);
      Fr[r] = qT ? (kf.y ^ kf.x) : kf.y;
    }
    if (lane == 0) Fr[0] |= pfix;
#pragma unroll
    for (int r = 0; r < kRows; r++) sh.hF[r][lane] = Fr[r];
    prim::wave_sync();
    uint32_t cc = base;
#pragma unroll 1
    for (uint32_t r = 0; r < R.head_rows; r++) {
      if constexpr (MIN) {
        // the kept bytes themselves: the row's segment is read again
        uint32_t w[8];
        load_segment<false>(a, P0 + (int64_t)r * kRowBytes + (int64_t)lane * kSegBytes, begin, end, w);
        write_bytes(sh, reinterpret_cast<uint8_t*>(a.out_idx) + S.hs, lim, &cc, sh.hF[r][lane], w);
      } else {
        write_row<(VAR & kVarDirectFlatten) == 0>(sh, out, lim, &cc, sh.hF[r][lane], rel0 + r * (uint32_t)kRowBytes);
      }
    }
    if (R.he_valid && lane == 0) {
      uint32_t err = 0;
      if (R.he_u | uT) err |= JSIDX_ERR_UTF8;
      if (R.he_R0 ^ qT) err |= JSIDX_ERR_UNCLOSED_STRING;
      if (R.he_EA) err |= JSIDX_ERR_TRAILING_ESCAPE;
      if (cc == 0) err |= JSIDX_ERR_EMPTY;
      prim::st_out(a.out_n + S.d_first + S.hd, cc);
      prim::st_out(a.out_err + S.d_first + S.hd, err);
    }
  }
  prim::trace(t, 7);
}

// ---------------------------------------------------------------------------
template <bool MIN = false, int VAR = 0>
JSIDX_DEV void index_tiles(const Args& a) {
  GroupShared& gs = prim::lds_object<GroupShared>();
  const uint32_t wv = prim::wave_id();
  Shared& sh = gs.w[wv];
  const uint32_t lane = prim::lane();
  Workspace* ws = a.ws;

  uint32_t epoch = 0;
  if (lane == 0) epoch = prim::ld_agent32(&ws->epoch);
  epoch = prim::readlane(epoch, 0);

  const int64_t begin = doc_off(a, 0);
  const int64_t end = doc_off(a, (int64_t)a.ndocs);
  const uintptr_t base_addr = (uintptr_t)a.base;
  const uintptr_t g0 = (base_addr + (uintptr_t)begin) & ~(uintptr_t)15;
  const int64_t pos_g0 = (int64_t)(g0 - base_addr);  // position of tile 0 byte 0
  const int64_t span = end - pos_g0;
  const uint32_t rows = a.rows ? a.rows : rows_for(span, a.fill_waves, a.rows_tab);
  const int64_t tb = (int64_t)rows * kRowBytes;
  const int64_t ntiles = span > 0 ? (span + tb - 1) / tb : 1;

  // offsets_check ran before this launch on the same stream (batches only)
  uint32_t bad = 0;
  if (a.offsets && lane == 0) bad = prim::ld_agent32(&ws->bad);
  bad = prim::readlane(bad, 0);
  if (bad || (uint64_t)ntiles > a.cap_tiles || (uint64_t)ntiles * rows > a.cap_rows) {
    // Not indexed: flag every document.  Nothing of the input is read.
    const uint32_t flag = bad ? JSIDX_ERR_OFFSETS : JSIDX_ERR_CAPACITY;
    for (int64_t d = ((int64_t)prim::block() * kWaves + wv) * kThreads + lane; d < a.ndocs;
         d += (int64_t)prim::grid() * kGroupThreads) {
      prim::st_out(a.out_n + d, 0u);
      prim::st_out(a.out_err + d, flag);
    }
  } else {
    // A ticket is tt consecutive tiles.  A workgroup takes its
    // waves' first tickets with one atomic (a launch starts thousands of
    // waves at once, and waves finishing together would otherwise queue on
    // one counter), then each wave takes tickets one at a time.  Tiles are
    // only ever handed to running waves, in increasing order.  A wave
    // finishes a tile (its look-back and head region) after the local pass
    // of its next tile, so that the look-back rarely waits; every tile
    // publishes before its wave waits for anything.
    const uint32_t tt = ntiles >= (int64_t)kTicketTiles * prim::grid() * kWaves ? (uint32_t)kTicketTiles : 1u;
    if (wv == 0 && lane == 0) gs.first = prim::add_agent32(&ws->ticket, (uint32_t)kWaves * tt);
    prim::sync();
    Pending pend;
    pend.valid = false;
    for (uint32_t tk = gs.first + wv * tt, left = tt;;) {
      const int64_t t = (int64_t)tk;
      if (t >= ntiles) break;
      prim::trace(t, 0);
      const TileSetup S = begin_tile(a, rows, sh, t, pos_g0, begin, end, ntiles);
      const Pending cur = start_tile<MIN, VAR>(a, sh, S, begin, end, ntiles, epoch);
      if (pend.valid) finish_tile<MIN, VAR>(a, sh, pend, pos_g0, begin, end, ntiles, epoch);
      pend = cur;
      tk++;
      if (--left == 0) {
        uint32_t nv = 0;
        if (lane == 0) nv = prim::add_agent32(&ws->ticket, tt);
        tk = prim::readlane(nv, 0);
        left = tt;
      }
    }
    if (pend.valid) finish_tile<MIN, VAR>(a, sh, pend, pos_g0, begin, end, ntiles, epoch);
  }

  // The last workgroup out resets the counters for the next launch and clears
  // a rotating window of descriptors so that no stale descriptor can ever
  // carry a matching epoch.
  prim::sync();
  if (wv == 0 && lane == 0) {
    prim::wait_mem();
    const uint32_t old = prim::add_agent32(&ws->done, 1u);
    gs.is_last = (old == prim::grid() - 1) ? 1u : 0u;
  }
  prim::sync();
  if (gs.is_last) {
    const uint64_t gl = (uint64_t)wv * kThreads + lane;
    const uint64_t nwin = (a.cap_tiles + kScrub - 1) / kScrub;
    const uint64_t w0 = (uint64_t)(epoch % (uint32_t)(nwin ? nwin : 1)) * kScrub;
    for (uint64_t j = w0 + gl; j < w0 + kScrub && j < a.cap_tiles; j += kGroupThreads) st_desc(ws, (int64_t)j, 0ull);
    for (uint64_t j = gl; j < 3 * blocks_for_tiles(a.cap_tiles); j += kGroupThreads) prim::st_agent(block_desc(a) + j, 0ull);
    prim::sync();
    if (wv == 0 && lane == 0) {
      prim::st_agent32(&ws->ticket, 0u);
      prim::st_agent32(&ws->done, 0u);
      prim::st_agent32(&ws->bad, 0u);
      prim::st_agent32(&ws->epoch, epoch + 1u);
    }
  }
}

// Before a batch launch: marks the workspace if offsets[d+1] < offsets[d] for
// some d (the indexing launch then flags every document instead of reading
// the input).  A grid-stride pass over the offsets.
JSIDX_DEVFN void offsets_check(const uint64_t* offsets, uint32_t ndocs, Workspace* ws, uint32_t threads) {
  uint32_t dec = 0;
  for (uint64_t d = (uint64_t)prim::block() * threads + prim::tid(); d < ndocs; d += (uint64_t)prim::grid() * threads)
    dec |= prim::load8(offsets + d + 1) < prim::load8(offsets + d) ? 1u : 0u;
  if (prim::ballot(dec != 0u) != 0ull && prim::lane() == 0) prim::or_agent32(&ws->bad, 1u);
}

}  // namespace jsidx
