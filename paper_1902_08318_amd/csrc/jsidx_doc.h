// jsidx_doc.h -- the stage-1 indexing kernel for ONE document (jsidx_build).
// Written against the primitives of jsidx_prims.h only.
//
// A wave owns a tile of kDocRows rows of 64 lanes x 32 bytes at a time and
// processes it in two passes:
//   local pass:  per row, the byte classes (Sec. 3.1.2), UTF-8 check
//                (Sec. 3.1.5), escapes (Fig. 3), string ranges (Fig. 4) and
//                the candidate and index masks of Fig. 5, assuming the tile
//                starts outside a string.  The masks K (candidates) and F0
//                (index if the tile starts outside a string) stay in the
//                wave's LDS; the tile publishes its string parity and its two
//                possible index counts.
//   finish pass: after the look-back has delivered the in-string state and
//                the index count before the tile, every row's index mask is
//                F0, or F0 ^ K inside a string (the formula of Fig. 5 is
//                symmetric in the string mask), and is flattened (Sec. 3.1.4).
// The escape and predecessor states entering a tile depend only on the bytes
// right before it (the backslash run ending there, and the class of the last
// byte), so the tile reads them itself; only the string parity and the count
// travel through the look-back.  A wave runs the local pass of its next tile
// before the finish pass of the current one, so look-backs rarely wait.
#pragma once
#include <stdint.h>

#include "jsidx.h"
#include "jsidx_device.h"
#include "jsidx_kernel.h"

namespace jsidx {

#ifndef JSIDX_DOC_ROWS
#define JSIDX_DOC_ROWS 8
#endif
constexpr int kDocRows = JSIDX_DOC_ROWS;            // rows per tile
constexpr int kDocTile = kDocRows * kRowBytes;      // 16 KiB
#ifndef JSIDX_DOC_WAVES
#define JSIDX_DOC_WAVES 12
#endif
constexpr int kDocWaves = JSIDX_DOC_WAVES;          // independent waves per workgroup
constexpr int kDocThreads = kDocWaves * kThreads;
#ifndef JSIDX_DOC_BLOCK
#define JSIDX_DOC_BLOCK 8
#endif
constexpr int kDocBlock = JSIDX_DOC_BLOCK;          // tiles per look-back block (<= 64)
constexpr int kDocScrub = 4096;                     // tile descriptors cleared per launch
// Tiles per batch: a workgroup claims kDocBatch consecutive tiles with one
// atomic on the global counter, and its waves take them one at a time from
// the workgroup's LDS pool (one counter hit by every wave per tile would
// serialize the launch on that counter).
#ifndef JSIDX_DOC_BATCH
#define JSIDX_DOC_BATCH 12
#endif
constexpr uint32_t kDocBatch = JSIDX_DOC_BATCH;
static_assert(kDocBatch >= 1 && kDocBatch < 128, "batch size fits the pool's count field");
// A batch's later tiles would start only after their wave waited for an
// earlier one, a chain through every batch: one tile per wave at most.
static_assert(kDocBatch <= kDocWaves, "a batch holds at most one tile per wave of the workgroup");
constexpr int kDocStage = kDocRows * kThreads * 2;  // uint32 entries of a tile's mask slot
// Mask slots per wave: a wave finishes a tile kDocSlots - 1 local passes
// after publishing it, so its look-back rarely waits for a slower tile.
#ifndef JSIDX_DOC_SLOTS
#define JSIDX_DOC_SLOTS 3
#endif
constexpr int kDocSlots = JSIDX_DOC_SLOTS;
static_assert(kDocSlots >= 2 && kDocSlots <= 4, "mask slots per wave");
// A row is written through LDS (coalesced stores, four positions per lane and
// store) when some lane holds more than this many positions; otherwise each
// lane stores its own.
#ifndef JSIDX_DOC_STAGE_LANE
#define JSIDX_DOC_STAGE_LANE 5
#endif
static_assert(kDocBlock >= 1 && kDocBlock <= 64, "a block is read by one wave");
static_assert(kDocTile <= 32768, "tile counts fit in 15 bits");

// ---- workspace ---------------------------------------------------------------
// The stream workspace (jsidx_kernel.h) is followed by this kernel's region:
// tile descriptors, two words per block (aggregate, inclusive) and one 32-bit
// counter per block.  The header (ticket, done, epoch, diag) is shared.
inline constexpr uint64_t doc_cap_for(uint64_t tiles16) { return tiles16 * (uint64_t)(kTileBytes / kDocTile) + 1; }
inline constexpr uint64_t doc_blocks_for(uint64_t cap) { return (cap + kDocBlock - 1) / kDocBlock; }
inline constexpr uint64_t doc_region_offset(uint64_t tiles16) { return (workspace_bytes(tiles16) + 255) & ~(uint64_t)255; }
inline constexpr uint64_t doc_region_bytes(uint64_t tiles16) {
  return doc_cap_for(tiles16) * 8 + doc_blocks_for(doc_cap_for(tiles16)) * 20 + 64;
}
// Everything a stream's workspace holds (both indexing kernels).
inline constexpr uint64_t stream_ws_bytes(uint64_t tiles16) {
  return doc_region_offset(tiles16) + doc_region_bytes(tiles16);
}

// ---- descriptors ---------------------------------------------------------------
// Tile descriptor, 64 bits:
//   0..1  flag: 0 none, 1 aggregate, 2 inclusive
//   2     aggregate: parity of the tile's unescaped quotes; inclusive: in a string after the tile
//   3     a UTF-8 error (aggregate: in the tile; inclusive: in the document so far)
//   4     the escape state after the tile is known (5: its value)
//   6     the tile's last byte is structural, white space or an unescaped quote
//   7..21 aggregate: index count if the tile starts outside a string;
//   22..36          ... if it starts inside one
//   7..38 inclusive: index count of the document up to the tile's end
//   39..63 launch epoch (25 bits)
constexpr uint32_t kDocEpochShift = 39;
constexpr uint64_t kDocEpochMask = (1ull << 25) - 1;
JSIDX_DEV uint64_t doc_epoch_bits(uint32_t epoch) { return ((uint64_t)epoch & kDocEpochMask) << kDocEpochShift; }
JSIDX_DEV bool doc_current(uint64_t d, uint32_t epoch) {
  return (d >> kDocEpochShift) == ((uint64_t)epoch & kDocEpochMask) && (d & 3u) != 0u;
}
JSIDX_DEV uint64_t doc_side(uint32_t u, uint32_t ek, uint32_t eo, uint32_t po) {
  return ((uint64_t)(u & 1u) << 3) | ((uint64_t)(ek & 1u) << 4) | ((uint64_t)(eo & 1u) << 5) |
         ((uint64_t)(po & 1u) << 6);
}
JSIDX_DEV uint64_t doc_agg(uint32_t qf, uint32_t c0, uint32_t c1, uint64_t side, uint32_t epoch) {
  return 1ull | ((uint64_t)(qf & 1u) << 2) | side | ((uint64_t)(c0 & 0x7FFFu) << 7) | ((uint64_t)(c1 & 0x7FFFu) << 22) |
         doc_epoch_bits(epoch);
}
JSIDX_DEV uint64_t doc_inc(uint32_t q, uint32_t count, uint64_t side, uint32_t epoch) {
  return 2ull | ((uint64_t)(q & 1u) << 2) | side | ((uint64_t)count << 7) | doc_epoch_bits(epoch);
}
JSIDX_DEV uint32_t dd_flag(uint64_t d) { return (uint32_t)d & 3u; }
JSIDX_DEV uint32_t dd_q(uint64_t d) { return (uint32_t)(d >> 2) & 1u; }
JSIDX_DEV uint32_t dd_u(uint64_t d) { return (uint32_t)(d >> 3) & 1u; }
JSIDX_DEV uint32_t dd_ek(uint64_t d) { return (uint32_t)(d >> 4) & 1u; }
JSIDX_DEV uint32_t dd_eo(uint64_t d) { return (uint32_t)(d >> 5) & 1u; }
JSIDX_DEV uint32_t dd_po(uint64_t d) { return (uint32_t)(d >> 6) & 1u; }
JSIDX_DEV uint32_t dd_c0(uint64_t d) { return (uint32_t)(d >> 7) & 0x7FFFu; }
JSIDX_DEV uint32_t dd_c1(uint64_t d) { return (uint32_t)(d >> 22) & 0x7FFFu; }
JSIDX_DEV uint32_t dd_count(uint64_t d) { return (uint32_t)(d >> 7); }

// Block words (cleared at the end of every launch, so no epoch):
//   aggregate: 1 | q flip << 2 | u << 3 | C0 << 4 (30 bits) | C1 << 34 (30 bits),
//              set by an atomic OR; bit 1 (kBlkPrev) is ORed in by the chain of
//              inclusive values when it reaches the block (see doc_chain)
//   inclusive: 2 | q << 2 | u << 3 | count << 4
JSIDX_DEV uint64_t blk_agg(uint32_t qf, uint32_t u, uint32_t c0, uint32_t c1) {
  return 1ull | ((uint64_t)qf << 2) | ((uint64_t)u << 3) | ((uint64_t)(c0 & 0x3FFFFFFFu) << 4) |
         ((uint64_t)(c1 & 0x3FFFFFFFu) << 34);
}
JSIDX_DEV uint64_t blk_inc(uint32_t q, uint32_t u, uint32_t count) {
  return 2ull | ((uint64_t)q << 2) | ((uint64_t)u << 3) | ((uint64_t)count << 4);
}
constexpr uint64_t kBlkPrev = 2ull;

struct DocArgs {
  const uint8_t* base;  // the document: base[0 .. len)
  uint64_t len;
  uint32_t* out_idx;
  uint32_t* out_n;
  uint32_t* out_err;
  Workspace* ws;        // shared header
  uint64_t* desc;       // cap tile descriptors
  uint64_t* blk;        // 2 words per block
  uint32_t* bcnt;       // 1 counter per block
  uint64_t cap;         // tile descriptors available
  int64_t p0;           // document position of tile 0's first byte: -(base mod 16)
  int64_t ntiles;
};

// Per-wave LDS: the masks (K, F0) of two tiles, one in its local pass and one
// waiting for its finish pass; a finishing tile's slot doubles as the
// flatten staging buffer once its masks are in registers.
struct alignas(16) DocWaveShared {
  uint2 m[kDocSlots][kDocRows][kThreads];
};
struct DocGroupShared {
  DocWaveShared w[kDocWaves];
  uint32_t pool;     // the workgroup's current batch of tiles: batch << 8 | tiles taken
  uint32_t is_last;
};

// Carries between rows (wave-uniform).
struct RowCarry {
  uint32_t e, q, p, u;  // escape, in-string, predecessor class, UTF-8 error seen
  U8Carry uc;
};

// What the local pass learned about a tile (wave-uniform).
struct DocTile {
  int64_t t, P0;
  uint32_t slot;
  uint32_t qpar, u, c0, c1;  // string parity, UTF-8 error, counts outside / inside
  uint32_t eo, ek, po;       // escape state after the tile (known?), class of its last byte
  uint32_t tesc;             // the document's last byte ends an odd backslash run
  uint32_t lead_q;           // the first byte that is not a backslash is a quote
  uint32_t lead_pos;         // ... at this tile position (kDocTile: none)
};

// ---- the bytes just before a tile ---------------------------------------------
struct Behind {
  uint32_t e, p;             // escape state entering byte P0, class of byte P0 - 1
  uint32_t e_known, p_known;
  U8Carry uc;                // UTF-8 state after byte P0 - 1
};

JSIDX_DEV bool is_cw(uint32_t b) {
  return b == 0x2Cu || b == 0x3Au || b == 0x5Bu || b == 0x5Du || b == 0x7Bu || b == 0x7Du || b == 0x20u ||
         b == 0x09u || b == 0x0Au || b == 0x0Du;
}

// The bytes just before a tile: lane i loads byte P0 - 1 - i (P0 >= 64,
// inside the document).  Issued before the tile's first row loads, so that
// waiting for it never waits for them.
JSIDX_DEV uint32_t rb_load(const DocArgs& a, int64_t P0) {
  return prim::load1(a.base + P0 - 1 - (int64_t)prim::lane());
}

// The escape state entering the tile is the parity of the backslash run
// ending at P0 - 1; the predecessor class is that of byte P0 - 1 (a quote
// counts if the run before it is even).  Runs of 64 or more leave the state
// unknown here.
JSIDX_DEV Behind rb_eval(uint32_t b) {
  const uint64_t BS = prim::ballot(b == 0x5Cu);
  Behind r;
  const uint32_t b0 = prim::readlane(b, 0), b1 = prim::readlane(b, 1), b2 = prim::readlane(b, 2),
                 b3 = prim::readlane(b, 3);
  r.uc = u8_carry_from_word(b3 | (b2 << 8) | (b1 << 16) | (b0 << 24));
  const uint64_t nbs = ~BS;
  r.e_known = nbs != 0ull;
  r.e = r.e_known ? ((uint32_t)__builtin_ctzll(nbs) & 1u) : 0u;
  r.p_known = 1;
  if (b0 == 0x22u) {
    const uint64_t nb2 = ~(BS >> 1) & (~0ull >> 1);
    r.p_known = nb2 != 0ull;
    r.p = ((uint32_t)__builtin_ctzll(nb2 | (1ull << 63)) & 1u) ^ 1u;  // even run: the quote is not escaped
  } else {
    r.p = is_cw(b0) ? 1u : 0u;
  }
  return r;
}

JSIDX_DEV Behind read_behind(const DocArgs& a, int64_t P0) { return rb_eval(rb_load(a, P0)); }

// This lane's 32 bytes at document position pos (pos is 16-byte aligned
// relative to the buffer).  Granules outside the document's granules are
// read from the granule holding byte 0 instead (their bytes are masked).
template <bool EDGE>
JSIDX_DEV void doc_load(const DocArgs& a, int64_t pos, uint32_t w[8]) {
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int64_t g = pos + 16 * h;
    const bool ok = !EDGE || (g < (int64_t)a.len && g + 16 > 0);
    const uint4 v = prim::load16(ok ? a.base + g : a.base + a.p0);
    w[4 * h + 0] = v.x; w[4 * h + 1] = v.y; w[4 * h + 2] = v.z; w[4 * h + 3] = v.w;
  }
}

// ---- one row of the local pass ----------------------------------------------------
// EDGE: the row holds bytes outside the document (before byte 0 or at or past
// len): they are masked to zero bytes, byte 0 gets a virtual white-space
// predecessor, and a sequence still open at the last byte is a UTF-8 error.
// The UTF-8 check of one row (Sec. 3.1.5), on values: the carry state comes
// in as cin and leaves in *cout; returns the error bits.  (The carries are
// kept in locals so that none of them ends up in private memory.)
JSIDX_DEV uint32_t doc_utf8(const uint32_t p[8], uint32_t D, uint32_t E, U8Carry cin, U8Carry* cout) {
  uint32_t l4 = cin.l4, x = cin.x, pa = cin.pa, m1c = cin.m1, m2c = cin.m2, m3c = cin.m3;
  const uint32_t cont = p[7] & ~p[6];
  const uint32_t lead = p[7] & p[6];
  const uint32_t L3 = lead & p[5];
  const uint32_t L4 = L3 & p[4];
  const uint32_t A1 = shift_in1(L4, &l4) & ~D;        // a 4-byte lead one back
  const uint32_t A2 = shift_in1(L3 | A1, &x) & ~D;    // 3+ lead one back or 4-byte two back
  const uint32_t PA = lead | A2;                      // the next byte must continue
  const uint32_t need = shift_in1(PA, &pa) & ~D;
  uint32_t err = (cont ^ need) | (PA & E);
  err |= lead & ~(p[5] | p[4] | p[3] | p[2] | p[1]);  // C0, C1
  err |= L4 & (p[3] | (p[2] & (p[1] | p[0])));        // F5..FF
  const uint32_t lowz = ~(p[3] | p[2] | p[1] | p[0]);
  const uint32_t x3 = L3 & ~p[4];                     // E0..EF
  const uint32_t E0 = x3 & lowz;
  const uint32_t ED = x3 & p[3] & p[2] & ~p[1] & p[0];
  const uint32_t F0 = L4 & lowz;
  const uint32_t F4 = L4 & ~p[3] & p[2] & ~p[1] & ~p[0];
  const uint32_t m1 = shift_in1(E0 | F0, &m1c) & ~D;  // low second bytes are errors
  const uint32_t m2 = shift_in1(ED | F4, &m2c) & ~D;  // high second bytes are errors
  const uint32_t m3 = shift_in1(F0 | F4, &m3c) & ~D;  // 4-byte lead: the bound is 0x90
  const uint32_t hi4 = m3 & p[4];
  err |= (m1 & ~p[5] & ~hi4) | (m2 & (p[5] | hi4));
  cout->l4 = l4; cout->x = x; cout->pa = pa; cout->m1 = m1c; cout->m2 = m2c; cout->m3 = m3c;
  return err;
}

// ---- one row of the local pass ----------------------------------------------------
// EDGE: the row holds bytes outside the document (before byte 0 or at or past
// len): they are masked to zero bytes, byte 0 gets a virtual white-space
// predecessor, and a sequence still open at the last byte is a UTF-8 error.
template <bool EDGE, int VAR>
JSIDX_DEV void doc_row(const DocArgs& a, const uint32_t w[8], int64_t pos, RowCarry& c, uint2* mrow,
                       uint32_t& a0, uint32_t& a1, DocTile& T, uint32_t rowpos, bool track_lead) {
  const uint32_t lane = prim::lane();
  uint32_t ce = c.e, cq = c.q, cp = c.p, cu = c.u;
  uint32_t V = ~0u, D = 0u, E = 0u;
  if constexpr (EDGE) {
    const int64_t vlo = -pos, vhi = (int64_t)a.len - pos;
    V = ge_mask((uint32_t)(vlo < 0 ? 0 : (vlo > 32 ? 32 : vlo))) & lt_mask((uint32_t)(vhi < 0 ? 0 : (vhi > 32 ? 32 : vhi)));
    if (pos <= 0 && pos > -32) D = 1u << (uint32_t)(-pos);
    const int64_t last = (int64_t)a.len - 1 - pos;
    if (last >= 0 && last < 32) E = 1u << (uint32_t)last;
  }
  ClassMasks cm;
  if constexpr ((VAR & kVarNaiveClassify) != 0) {
    SegWords sw;
#pragma unroll
    for (int k = 0; k < 8; k++) sw.w[k] = w[k];
    cm = classify_bytes(sw);
  }
  uint32_t pl[8];
  bit_planes(w, pl);
  if constexpr (EDGE) {
#pragma unroll
    for (int k = 0; k < 8; k++) pl[k] &= V;
  }
  if constexpr ((VAR & kVarNaiveClassify) != 0) {
    if constexpr (EDGE) { cm.C &= V; cm.W &= V; cm.Q &= V; cm.B &= V; }
  } else {
    cm = classify_planes(pl);
  }

  // UTF-8: rows without a byte >= 0x80 and with no sequence open from the
  // row before have no errors
  U8Carry uc;
  if (prim::ballot(pl[7] != 0u) != 0ull || u8_carry_pending(c.uc)) {
    const uint32_t errm = doc_utf8(pl, D, E, c.uc, &uc);
    if (prim::ballot(errm != 0u) != 0ull) cu = 1u;
  } else {
    uc = u8_carry_zero();
  }
  c.uc = uc;

  // the first byte of the tile that is not a backslash (only needed when the
  // escape state entering the tile is not known from the bytes before it)
  if (track_lead && T.lead_pos == (uint32_t)kDocTile) {
    const uint64_t Kc = prim::ballot(cm.B != ~0u);
    if (Kc) {
      const int f = __builtin_ctzll(Kc);
      const uint32_t nb = ~cm.B;
      const uint32_t j = nb ? (uint32_t)__builtin_ctz(nb) : 0u;
      const uint32_t lp = rowpos + (uint32_t)f * (uint32_t)kSegBytes + prim::readlane(j, f);
      const uint32_t lq = prim::readlane((cm.Q >> j) & 1u, f);
      T.lead_pos = lp;
      T.lead_q = lq;
    }
  }

  // escapes (Fig. 3): the escape entering each lane is the parity of the
  // backslash run ending the lanes before (a lane of 32 backslashes passes it
  // on unchanged)
  uint32_t OD;
  uint32_t e_lane = 0;
  if (prim::ballot(cm.B != 0u) == 0ull) {
    e_lane = lane == 0 ? ce : 0u;
    OD = e_lane;
    ce = 0u;
  } else {
    const uint32_t nb = ~cm.B;
    const uint32_t eo = (nb ? (uint32_t)__builtin_clz(nb) : 32u) & 1u;  // the trailing run is odd
    if (prim::ballot(cm.B == ~0u) == 0ull) {
      e_lane = shift_in1(eo << 31, &ce) & 1u;
    } else {
      const uint64_t Kc = prim::ballot(cm.B != ~0u);
      const uint64_t Ec = prim::ballot(eo != 0u && cm.B != ~0u);
      const uint64_t mk = Kc & lt_lanes();
      e_lane = mk ? (uint32_t)((Ec >> msb64(mk)) & 1ull) : ce;
      if (Kc) ce = (uint32_t)((Ec >> msb64(Kc)) & 1ull);
    }
    OD = odd_run_ends(cm.B & ~e_lane) | e_lane;
  }
  const uint32_t Q = cm.Q & ~OD;

  // string ranges (Fig. 4): prefix XOR inside the lane, the parity of the
  // lanes before by ballot
  const uint32_t PX = (VAR & kVarXorLoop) ? prefix_xor_loop(Q) : prefix_xor(Q);
  const uint64_t Qb = prim::ballot((__builtin_popcount(Q) & 1u) != 0u);
  const uint32_t qin = (prim::mbcnt(Qb) & 1u) ^ cq;
  const uint32_t R0 = PX ^ (0u - qin);
  cq ^= parity64(Qb);

  // structural and pseudo-structural bytes (Fig. 5)
  const uint32_t P0m = cm.C | cm.W | Q;
  uint32_t PR = shift_in1(P0m, &cp);
  if constexpr (EDGE) PR |= D;
  uint32_t K = cm.C | Q | (PR & ~P0m);
  if constexpr (EDGE) K &= V;
  const uint32_t F0 = K & ~(Q ^ R0);
  uint2 kf;
  kf.x = K;
  kf.y = F0;
  mrow[lane] = kf;
  a0 += (uint32_t)__builtin_popcount(F0);
  a1 += (uint32_t)__builtin_popcount(F0 ^ K);

  if constexpr (EDGE) {
    // the escape state after the document's last byte: the escape of the
    // byte after it (a masked zero byte in this lane), or what the lane
    // passes on
    if (prim::ballot(E != 0u) != 0ull) {
      const int64_t nx = (int64_t)a.len - pos;  // position of the byte after the last, in this lane
      const uint32_t e_next = prim::shfl(e_lane, (int)((lane + 1u) & 63u));
      uint32_t te = 0;
      if (E != 0u) te = nx < 32 ? (OD >> (uint32_t)nx) & 1u : (lane == 63 ? ce : e_next);
      T.tesc = prim::readlane(te, __builtin_ctzll(prim::ballot(E != 0u)));
    }
  }
  c.e = ce; c.q = cq; c.p = cp; c.u = cu;
}

// ---- one interior row, carries by lane rotation -------------------------------------
// Every 1-bit shift that crosses a lane boundary, (x << 1) with bit 0 from bit
// 31 of the lane before, takes the lane before's x by one DPP wave rotation;
// lane 0 takes it from the previous row's rotation, kept in a register
// (`rot`, valid in lane 0), so no carry goes through scalar registers.
JSIDX_DEV uint32_t shl1_rot(uint32_t x, uint32_t& rot, bool lane0) {
  const uint32_t r = prim::ror1(x);
  const uint32_t prev = lane0 ? rot : r;
  rot = r;
  return prim::alignbit(x, prev, 31);
}

// Carries between the interior rows of a tile.
struct FastCarry {
  uint32_t rp;          // predecessor class (bit 31, lane 0)
  uint32_t ru[6];       // UTF-8: 4-byte lead, 3+ lead, continuation needed, E0|F0, ED|F4, F0|F4
  uint32_t e, q, u;     // escape, in-string, UTF-8 error seen (uniform)
  uint32_t u8pend;      // a multi-byte sequence is open at the end of the previous row (uniform)
};

JSIDX_DEV void fast_carry_from(FastCarry& f, const Behind& B) {
  f.rp = B.p << 31;
  f.ru[0] = B.uc.l4 << 31; f.ru[1] = B.uc.x << 31; f.ru[2] = B.uc.pa << 31;
  f.ru[3] = B.uc.m1 << 31; f.ru[4] = B.uc.m2 << 31; f.ru[5] = B.uc.m3 << 31;
  f.e = B.e; f.q = 0u; f.u = 0u;
  f.u8pend = u8_carry_pending(B.uc) ? 1u : 0u;
}

template <int VAR>
JSIDX_DEV void doc_row_fast(const uint32_t w[8], FastCarry& c, uint2* mrow, uint32_t& a0, uint32_t& a1, DocTile& T,
                            uint32_t rowpos, bool track_lead) {
  const uint32_t lane = prim::lane();
  const bool l0 = lane == 0u;
  ClassMasks cm;
  if constexpr ((VAR & kVarNaiveClassify) != 0) {
    SegWords sw;
#pragma unroll
    for (int k = 0; k < 8; k++) sw.w[k] = w[k];
    cm = classify_bytes(sw);
  }
  uint32_t pl[8];
  bit_planes(w, pl);
  if constexpr ((VAR & kVarNaiveClassify) == 0) cm = classify_planes(pl);

  // UTF-8 (Sec. 3.1.5): a byte is a continuation exactly where a lead one,
  // two or three bytes back asks for one; C0, C1, F5..FF never occur; the
  // byte after E0 / ED / F0 / F4 is range checked.  Rows without a byte >=
  // 0x80 and with nothing open from the row before skip it (their carries
  // are then zero, and so are the rotations' bits read later).
  if (prim::ballot(pl[7] != 0u) != 0ull || c.u8pend) {
    const uint32_t p7 = pl[7], p6 = pl[6], p5 = pl[5], p4 = pl[4];
    const uint32_t cont = p7 & ~p6;
    const uint32_t lead = p7 & p6;
    const uint32_t L3 = lead & p5;
    const uint32_t L4 = L3 & p4;
    const uint32_t A1 = shl1_rot(L4, c.ru[0], l0);
    const uint32_t A2 = shl1_rot(L3 | A1, c.ru[1], l0);
    const uint32_t PA = lead | A2;
    const uint32_t need = shl1_rot(PA, c.ru[2], l0);
    uint32_t err = cont ^ need;
    err |= lead & ~(p5 | p4 | pl[3] | pl[2] | pl[1]);        // C0, C1
    err |= L4 & (pl[3] | (pl[2] & (pl[1] | pl[0])));         // F5..FF
    const uint32_t lowz = ~(pl[3] | pl[2] | pl[1] | pl[0]);
    const uint32_t x3 = L3 & ~p4;                            // E0..EF
    const uint32_t E0 = x3 & lowz;
    const uint32_t ED = x3 & pl[3] & pl[2] & ~pl[1] & pl[0];
    const uint32_t F0 = L4 & lowz;
    const uint32_t F4 = L4 & ~pl[3] & pl[2] & ~pl[1] & ~pl[0];
    const uint32_t m1 = shl1_rot(E0 | F0, c.ru[3], l0);      // low second bytes are errors
    const uint32_t m2 = shl1_rot(ED | F4, c.ru[4], l0);      // high second bytes are errors
    const uint32_t m3 = shl1_rot(F0 | F4, c.ru[5], l0);      // 4-byte lead: the bound is 0x90
    const uint32_t hi4 = m3 & p4;
    err |= (m1 & ~p5 & ~hi4) | (m2 & (p5 | hi4));
    if (prim::ballot(err != 0u) != 0ull) c.u = 1u;
    // open at the row's end: bit 31 of a lead-derived mask in lane 63
    c.u8pend = prim::readlane(L4 | (L3 | A1) | PA, 63) >> 31;
  }

  if (track_lead && T.lead_pos == (uint32_t)kDocTile) {
    const uint64_t Kc = prim::ballot(cm.B != ~0u);
    if (Kc) {
      const int f = __builtin_ctzll(Kc);
      const uint32_t nb = ~cm.B;
      const uint32_t j = nb ? (uint32_t)__builtin_ctz(nb) : 0u;
      T.lead_pos = rowpos + (uint32_t)f * (uint32_t)kSegBytes + prim::readlane(j, f);
      T.lead_q = prim::readlane((cm.Q >> j) & 1u, f);
    }
  }

  // escapes (Fig. 3)
  uint32_t OD;
  if (prim::ballot(cm.B != 0u) == 0ull) {
    OD = l0 ? c.e : 0u;
    c.e = 0u;
  } else {
    const uint32_t nb = ~cm.B;
    const uint32_t eo = (nb ? (uint32_t)__builtin_clz(nb) : 32u) & 1u;  // the trailing run is odd
    uint32_t e_lane;
    if (prim::ballot(cm.B == ~0u) == 0ull) {
      e_lane = prim::shr1(eo, c.e);
      c.e = prim::readlane(eo, 63);
    } else {
      const uint64_t Kc = prim::ballot(cm.B != ~0u);
      const uint64_t Ec = prim::ballot(eo != 0u && cm.B != ~0u);
      const uint64_t mk = Kc & lt_lanes();
      e_lane = mk ? (uint32_t)((Ec >> msb64(mk)) & 1ull) : c.e;
      if (Kc) c.e = (uint32_t)((Ec >> msb64(Kc)) & 1ull);
    }
    OD = odd_run_ends(cm.B & ~e_lane) | e_lane;
  }
  const uint32_t Q = cm.Q & ~OD;

  // string ranges (Fig. 4)
  const uint32_t PX = (VAR & kVarXorLoop) ? prefix_xor_loop(Q) : prefix_xor(Q);
  const uint64_t Qb = prim::ballot((__builtin_popcount(Q) & 1u) != 0u);
  const uint32_t qin = (prim::mbcnt(Qb) & 1u) ^ c.q;
  const uint32_t R0 = PX ^ (0u - qin);
  c.q ^= parity64(Qb);

  // structural and pseudo-structural bytes (Fig. 5)
  const uint32_t P0m = cm.C | cm.W | Q;
  const uint32_t PR = shl1_rot(P0m, c.rp, l0);
  const uint32_t K = cm.C | Q | (PR & ~P0m);
  const uint32_t F0 = K & ~(Q ^ R0);
  uint2 kf;
  kf.x = K;
  kf.y = F0;
  mrow[lane] = kf;
  a0 += (uint32_t)__builtin_popcount(F0);
  a1 += (uint32_t)__builtin_popcount(F0 ^ K);
}

// ---- the local pass over a tile ------------------------------------------------------
template <int VAR>
JSIDX_DEV void doc_local(const DocArgs& a, DocWaveShared& sh, DocTile& T, uint32_t e_in, uint32_t p_in, U8Carry uc,
                         bool track_lead) {
  const uint32_t lane = prim::lane();
  const int64_t P0 = T.P0;
  // a row or tile is treated as an edge if it holds bytes outside the document
  // or ends exactly at its end (the trailing escape is read there)
  const bool edge = P0 < 0 || P0 + kDocTile >= (int64_t)a.len;
  RowCarry c;
  c.e = e_in; c.q = 0u; c.p = p_in; c.u = 0u; c.uc = uc;
  uint32_t a0 = 0, a1 = 0;
  T.tesc = 0; T.lead_q = 0; T.lead_pos = (uint32_t)kDocTile;
  uint2(*m)[kThreads] = sh.m[T.slot];
  uint32_t wn[8];
  if (edge) doc_load<true>(a, P0 + (int64_t)lane * kSegBytes, wn);
  else doc_load<false>(a, P0 + (int64_t)lane * kSegBytes, wn);
#pragma unroll 1
  for (int r = 0; r < kDocRows; r++) {
    const int64_t pos = P0 + (int64_t)r * kRowBytes + (int64_t)lane * kSegBytes;
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; k++) w[k] = wn[k];
    const int64_t rp = P0 + (int64_t)r * kRowBytes;
    const bool row_edge = edge && (rp < 0 || rp + kRowBytes >= (int64_t)a.len);
    if (r + 1 < kDocRows) {
      if (edge) doc_load<true>(a, pos + kRowBytes, wn);
      else doc_load<false>(a, pos + kRowBytes, wn);
    }
    if (row_edge) doc_row<true, VAR>(a, w, pos, c, m[r], a0, a1, T, (uint32_t)(r * kRowBytes), track_lead);
    else doc_row<false, VAR>(a, w, pos, c, m[r], a0, a1, T, (uint32_t)(r * kRowBytes), track_lead);
  }
  T.qpar = c.q;
  T.u = c.u;
  T.c0 = wave_sum(a0);
  T.c1 = wave_sum(a1);
  T.eo = c.e;
  T.po = c.p;
}

// The local pass over a tile that lies inside the document (no masking),
// rows unrolled, kDocAhead rows of loads in flight.  With B_IN false the
// state entering the tile is read from the bytes before it (the read-behind
// load goes out first) and returned in *B; otherwise *B is the state to use.
#ifndef JSIDX_DOC_AHEAD
#define JSIDX_DOC_AHEAD 2
#endif
constexpr int kDocAhead = JSIDX_DOC_AHEAD;
static_assert(kDocAhead >= 1 && kDocAhead <= kDocRows, "prefetch depth");

// Loads issued for a tile before its local pass: the bytes before it and its
// first kDocAhead rows (interior tiles only).
struct DocPre {
  uint32_t rb;
  uint32_t w[kDocAhead][8];
};

JSIDX_DEV void doc_prefetch(const DocArgs& a, int64_t P0, DocPre& S) {
  const uint8_t* src = a.base + P0 + (int64_t)prim::lane() * kSegBytes;
  S.rb = rb_load(a, P0);
#pragma unroll
  for (int p = 0; p < kDocAhead; p++) {
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const uint4 v = prim::load16(src + p * kRowBytes + 16 * h);
      S.w[p][4 * h + 0] = v.x; S.w[p][4 * h + 1] = v.y; S.w[p][4 * h + 2] = v.z; S.w[p][4 * h + 3] = v.w;
    }
  }
}

// The local pass over a tile that lies inside the document (no masking),
// rows unrolled, kDocAhead rows of loads in flight; S holds the prefetched
// bytes before the tile and its first rows.  With B_IN false the state
// entering the tile comes from S.rb and is returned in *B; otherwise *B is
// the state to use.
template <int VAR, bool B_IN>
JSIDX_DEV void doc_local_fast(const DocArgs& a, DocWaveShared& sh, DocTile& T, Behind* B, bool track_lead,
                              const DocPre& S) {
  const uint32_t lane = prim::lane();
  const uint8_t* src = a.base + T.P0 + (int64_t)lane * kSegBytes;
  uint32_t buf[kDocAhead][8];
#pragma unroll
  for (int p = 0; p < kDocAhead; p++)
#pragma unroll
    for (int k = 0; k < 8; k++) buf[p][k] = S.w[p][k];
  if constexpr (!B_IN) *B = rb_eval(S.rb);
  FastCarry c;
  fast_carry_from(c, *B);
  uint32_t a0 = 0, a1 = 0;
  T.tesc = 0; T.lead_q = 0; T.lead_pos = (uint32_t)kDocTile;
  uint2(*m)[kThreads] = sh.m[T.slot];
#pragma unroll
  for (int r = 0; r < kDocRows; r++) {
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; k++) w[k] = buf[r % kDocAhead][k];
    if (r + kDocAhead < kDocRows) {
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const uint4 v = prim::load16(src + (r + kDocAhead) * kRowBytes + 16 * h);
        buf[r % kDocAhead][4 * h + 0] = v.x; buf[r % kDocAhead][4 * h + 1] = v.y;
        buf[r % kDocAhead][4 * h + 2] = v.z; buf[r % kDocAhead][4 * h + 3] = v.w;
      }
    }
    doc_row_fast<VAR>(w, c, m[r], a0, a1, T, (uint32_t)(r * kRowBytes), track_lead);
  }
  T.qpar = c.q;
  T.u = c.u;
  T.c0 = wave_sum(a0);
  T.c1 = wave_sum(a1);
  T.eo = c.e;
  T.po = prim::readlane(c.rp, 0) >> 31;  // the class of the tile's last byte
}

// ---- the look-back -------------------------------------------------------------------
// A fold of consecutive tiles or blocks: either a known state (q, u, count)
// after them, or an aggregate (q flip, u, counts for an incoming q of 0 / 1).
struct DocFold {
  uint32_t known, pending;
  uint32_t q, u, c0, c1;  // known: q, u, c0 = count
};

// Folds descriptors held one per lane, lanes [0, n) in order (lane 0 the
// oldest): from the newest inclusive lane (or from `start` if none and
// start.known) over the aggregates after it.  Lanes with kind 0 are not yet
// published (pending).  kind / q / u / c0 / c1 per lane: 1 aggregate, 2
// inclusive (c0 = count).
JSIDX_DEV DocFold doc_fold(uint32_t kind, uint32_t q, uint32_t u, uint32_t c0, uint32_t c1, int n) {
  const uint32_t lane = prim::lane();
  const bool act = (int)lane < n;
  DocFold F;
  F.known = 0; F.pending = 0; F.q = 0; F.u = 0; F.c0 = 0; F.c1 = 0;
  const uint64_t Inc = prim::ballot(act && kind == 2u);
  const int k = Inc ? msb64(Inc) : -1;  // newest inclusive lane
  const uint64_t after = k >= 0 ? (~lanes_below(k + 1) & lanes_below(n)) : lanes_below(n);
  const uint64_t Pn = prim::ballot(act && kind == 0u) & after;
  if (Pn) { F.pending = 1; return F; }
  const bool in = ((after >> lane) & 1ull) != 0ull;
  const uint64_t Qf = prim::ballot(in && q != 0u);
  const uint32_t qb = prim::mbcnt(Qf) & 1u;  // flips of the lanes in `after` below this one
  const uint32_t Ua = prim::ballot(in && u != 0u) != 0ull;
  if (k >= 0) {
    const uint32_t kq = prim::readlane(q, k), ku = prim::readlane(u, k), kc = prim::readlane(c0, k);
    const uint32_t qe = kq ^ qb;
    const uint32_t s = wave_sum(in ? (qe ? c1 : c0) : 0u);
    F.known = 1;
    F.q = kq ^ parity64(Qf);
    F.u = ku | Ua;
    F.c0 = kc + s;
  } else {
    F.q = parity64(Qf);
    F.u = Ua;
    F.c0 = wave_sum(in ? (qb ? c1 : c0) : 0u);
    F.c1 = wave_sum(in ? (qb ? c0 : c1) : 0u);
  }
  return F;
}

// older then newer (newer is an aggregate)
JSIDX_DEV DocFold doc_then(const DocFold& older, const DocFold& newer) {
  DocFold r;
  r.pending = 0;
  if (older.known) {
    r.known = 1;
    r.c0 = older.c0 + (older.q ? newer.c1 : newer.c0);
    r.q = older.q ^ newer.q;
    r.u = older.u | newer.u;
    r.c1 = 0;
  } else {
    r.known = 0;
    r.c0 = older.c0 + (older.q ? newer.c1 : newer.c0);
    r.c1 = older.c1 + (older.q ? newer.c0 : newer.c1);
    r.q = older.q ^ newer.q;
    r.u = older.u | newer.u;
  }
  return r;
}

JSIDX_DEV void doc_poll_sleep(uint32_t polls) {
  const int n = polls < 2 ? 1 : (polls < 4 ? 2 : (polls < 8 ? 4 : 16));
  for (int i = 0; i < n; i++) prim::sleep();
}

// The state entering block b (b >= 1): the nearest block inclusive value before
// it, over the block aggregates after that.  Publishes block b-1's inclusive
// value when it had none.  Returns false if a wait gave up.
JSIDX_DEV bool doc_block_entry(const DocArgs& a, int64_t b, DocFold* out) {
  const uint32_t lane = prim::lane();
  DocFold acc;  // aggregate of the blocks after the window being read
  acc.known = 0; acc.pending = 0; acc.q = 0; acc.u = 0; acc.c0 = 0; acc.c1 = 0;
  bool have_acc = false;
  int64_t hi = b;  // blocks [hi - 64, hi) are read next
  for (uint32_t polls = 0;;) {
    const int64_t lo = hi - 64 > 0 ? hi - 64 : 0;
    const int n = (int)(hi - lo);
    const int64_t j = lo + (int64_t)lane;
    uint64_t inc = 0, agg = 0;
    if ((int)lane < n) {  // both words at once: one round trip
      agg = prim::ld_agent(a.blk + 2 * j);
      inc = prim::ld_agent(a.blk + 2 * j + 1);
    }
    uint32_t kind = 0, q = 0, u = 0, c0 = 0, c1 = 0;
    if ((inc & 3u) == 2u) {
      kind = 2; q = (uint32_t)(inc >> 2) & 1u; u = (uint32_t)(inc >> 3) & 1u; c0 = (uint32_t)(inc >> 4);
    } else if ((agg & 1u) != 0u) {
      kind = 1; q = (uint32_t)(agg >> 2) & 1u; u = (uint32_t)(agg >> 3) & 1u;
      c0 = (uint32_t)(agg >> 4) & 0x3FFFFFFFu; c1 = (uint32_t)(agg >> 34) & 0x3FFFFFFFu;
    }
    const DocFold F = doc_fold(kind, q, u, c0, c1, n);
    if (F.pending || (!F.known && lo == 0)) {
      // block 0 always ends known once published: wait
      if (++polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); return false; }
      doc_poll_sleep(polls);
      continue;
    }
    const DocFold whole = have_acc ? doc_then(F, acc) : F;
    if (whole.known) {
      // the state after block b - 1: publish it for the tiles still to come
      *out = whole;
      if (lane == 0) {
        const uint64_t cur = prim::ld_agent(a.blk + 2 * (b - 1) + 1);
        if ((cur & 3u) != 2u) prim::st_agent(a.blk + 2 * (b - 1) + 1, blk_inc(whole.q, whole.u, whole.c0));
      }
      return true;
    }
    acc = whole;  // 64 aggregates without an inclusive value: go further back
    have_acc = true;
    hi = lo;
    polls = 0;
  }
}

// The look-back's first reads, issued early (a local pass before they are
// needed, so that their round trip overlaps it): the descriptors of the
// tiles of t's block before t, one per lane, and the inclusive value of the
// block before (lane 0).
struct LbPre {
  uint64_t d, be;
};

JSIDX_DEV void doc_lb_issue(const DocArgs& a, int64_t t, LbPre& P) {
  const uint32_t lane = prim::lane();
  const int64_t b = t / kDocBlock, j0 = b * kDocBlock;
  P.d = 0;
  P.be = 0;
  if ((int64_t)lane < t - j0) P.d = prim::ld_agent(a.desc + j0 + lane);
  if (b > 0 && lane == 0) P.be = prim::ld_agent(a.blk + 2 * (b - 1) + 1);
}

// State entering tile t (t >= 1): q, u and the index count before it.  pre:
// the first reads, issued earlier (they may be stale; anything not yet
// published is read again).
JSIDX_DEV bool doc_look_back(const DocArgs& a, int64_t t, uint32_t epoch, DocFold* out, const LbPre* pre) {
  const uint32_t lane = prim::lane();
  const int64_t b = t / kDocBlock, j0 = b * kDocBlock;
  const int n = (int)(t - j0);
  bool have_entry = b == 0;
  DocFold entry;
  entry.known = 1; entry.pending = 0; entry.q = 0; entry.u = 0; entry.c0 = 0; entry.c1 = 0;
  for (uint32_t polls = 0;;) {
    uint64_t d = 0, be = 0;
    if (polls == 0 && pre) {
      d = pre->d;
      be = pre->be;
    } else {
      if ((int)lane < n) d = prim::ld_agent(a.desc + j0 + lane);
      if (!have_entry && lane == 0) be = prim::ld_agent(a.blk + 2 * (b - 1) + 1);
    }
    const bool ok = (int)lane < n && doc_current(d, epoch);
    const uint32_t kind = ok ? dd_flag(d) : 0u;
    const uint32_t q = dd_q(d), u = dd_u(d);
    const uint32_t c0 = kind == 2u ? dd_count(d) : dd_c0(d), c1 = dd_c1(d);
    DocFold F = doc_fold(kind, q, u, c0, c1, n);
    if (F.pending) {
      prim::dcount(t, 1u);
      if (++polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); return false; }
      doc_poll_sleep(polls);
      continue;
    }
    if (F.known) { *out = F; return true; }
    // no inclusive tile in this block before t: the state entering the block
    if (!have_entry) {
      const uint32_t blo = prim::readlane((uint32_t)be, 0), bhi = prim::readlane((uint32_t)(be >> 32), 0);
      const uint64_t bv = ((uint64_t)bhi << 32) | blo;
      if ((bv & 3u) == 2u) {
        entry.q = (uint32_t)(bv >> 2) & 1u; entry.u = (uint32_t)(bv >> 3) & 1u; entry.c0 = (uint32_t)(bv >> 4);
      } else {
        prim::dcount(t, 1u << 8);
        if (!doc_block_entry(a, b, &entry)) return false;
      }
    }
    *out = n == 0 ? entry : doc_then(entry, F);
    return true;
  }
}

// The chain of block inclusive values.  With the state after block x - 1
// known (E), it publishes the inclusive values of blocks x, x + 1, ... whose
// aggregates are in, 64 blocks per read (a scan over the lanes), and stops at
// the first block without one, handing the chain over: it ORs kBlkPrev into
// that block's aggregate word, and that block's fold ORs its aggregate into
// the same word; whichever of the two comes second (it sees the other's bit)
// continues the chain, so exactly one does, and the block inclusive values
// follow the folds closely.
JSIDX_DEV DocFold blk_state_agg(uint64_t w) {
  DocFold F;
  F.known = 0; F.pending = 0;
  F.q = (uint32_t)(w >> 2) & 1u; F.u = (uint32_t)(w >> 3) & 1u;
  F.c0 = (uint32_t)(w >> 4) & 0x3FFFFFFFu; F.c1 = (uint32_t)(w >> 34) & 0x3FFFFFFFu;
  return F;
}

JSIDX_DEV void doc_chain(const DocArgs& a, int64_t x, DocFold E) {
  const uint32_t lane = prim::lane();
  const int64_t nb = (a.ntiles + kDocBlock - 1) / kDocBlock;
  while (x < nb) {
    const int64_t j = x + (int64_t)lane;
    uint64_t w = 0;
    if (j < nb) w = prim::ld_agent(a.blk + 2 * j);
    const uint64_t ready = prim::ballot(j < nb && (w & 1ull) != 0ull);
    const int g = ~ready ? (int)__builtin_ctzll(~ready) : 64;  // blocks [x, x + g) are in
    if (g > 0) {
      const bool in = (int)lane < g;
      const DocFold A = blk_state_agg(w);
      const uint32_t q_in = E.q ^ (prim::mbcnt(prim::ballot(in && A.q != 0u)) & 1u);
      const uint32_t cnt = E.c0 + prim::incl_scan(in ? (q_in ? A.c1 : A.c0) : 0u);
      const uint32_t qo = q_in ^ A.q;
      const uint32_t uo = E.u | ((prim::ballot(in && A.u != 0u) & lanes_below((int)lane + 1)) != 0ull ? 1u : 0u);
      if (in) prim::st_agent(a.blk + 2 * j + 1, blk_inc(qo, uo, cnt));
      E.q = prim::readlane(qo, g - 1);
      E.u = prim::readlane(uo, g - 1);
      E.c0 = prim::readlane(cnt, g - 1);
      x += g;
    }
    if (g == 64 || x >= nb) continue;
    uint64_t old = 0;
    if (lane == 0) old = prim::or_agent64(a.blk + 2 * x, kBlkPrev);
    const uint32_t olo = prim::readlane((uint32_t)old, 0), ohi = prim::readlane((uint32_t)(old >> 32), 0);
    old = ((uint64_t)ohi << 32) | olo;
    if ((old & 1ull) == 0ull || (old & kBlkPrev) != 0ull) return;  // the block's fold continues
    E = doc_then(E, blk_state_agg(old));
    if (lane == 0) prim::st_agent(a.blk + 2 * x + 1, blk_inc(E.q, E.u, E.c0));
    x += 1;
  }
}

// The last tile of a block to publish folds the block's tile descriptors:
// it publishes the block's inclusive value if a tile of the block already
// has one (and carries the chain on from there), else ORs the aggregate into
// the block's aggregate word, and carries the chain on if it had reached the
// block.
JSIDX_DEV void doc_fold_block(const DocArgs& a, int64_t b, uint32_t epoch, int64_t t) {
  const uint32_t lane = prim::lane();
  const int64_t j0 = b * kDocBlock;
  const int64_t n64 = a.ntiles - j0 < kDocBlock ? a.ntiles - j0 : kDocBlock;
  const int n = (int)n64;
  DocFold F;
  for (uint32_t polls = 0;;) {
    uint64_t d = 0;
    if ((int)lane < n) d = prim::ld_agent(a.desc + j0 + lane);
    const bool ok = (int)lane < n && doc_current(d, epoch);
    const uint32_t kind = ok ? dd_flag(d) : 0u;
    F = doc_fold(kind, dd_q(d), dd_u(d), kind == 2u ? dd_count(d) : dd_c0(d), dd_c1(d), n);
    if (!F.pending) break;
    // a descriptor whose store is still on its way reads as not published:
    // read again
    prim::dcount(t, 1ull << 16);
    if (++polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); return; }
    doc_poll_sleep(polls);
  }
  if (F.known) {
    if (lane == 0) prim::st_agent(a.blk + 2 * b + 1, blk_inc(F.q, F.u, F.c0));
    doc_chain(a, b + 1, F);
    return;
  }
  uint64_t old = 0;
  if (lane == 0) old = prim::or_agent64(a.blk + 2 * b, blk_agg(F.q, F.u, F.c0, F.c1));
  if ((prim::readlane((uint32_t)old, 0) & (uint32_t)kBlkPrev) == 0u) return;
  // the chain is waiting here: the block before has its inclusive value
  // (stored before the chain's OR; read until it shows)
  DocFold E;
  for (uint32_t polls = 0;;) {
    uint64_t pv = 0;
    if (lane == 0) pv = prim::ld_agent(a.blk + 2 * (b - 1) + 1);
    const uint32_t plo = prim::readlane((uint32_t)pv, 0), phi = prim::readlane((uint32_t)(pv >> 32), 0);
    pv = ((uint64_t)phi << 32) | plo;
    if ((pv & 3u) == 2u) {
      E.known = 1; E.pending = 0; E.q = (uint32_t)(pv >> 2) & 1u; E.u = (uint32_t)(pv >> 3) & 1u;
      E.c0 = (uint32_t)(pv >> 4); E.c1 = 0;
      break;
    }
    if (++polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); return; }
    doc_poll_sleep(polls);
  }
  const DocFold W = doc_then(E, F);
  if (lane == 0) prim::st_agent(a.blk + 2 * b + 1, blk_inc(W.q, W.u, W.c0));
  doc_chain(a, b + 1, W);
}

// The escape state entering tile t when the bytes before it are 64 or more
// backslashes: the escape state after the newest earlier tile that knows it
// (tiles in between are all backslashes, an even number, so they pass it on).
JSIDX_DEV bool doc_escape_walk(const DocArgs& a, int64_t t, uint32_t epoch, uint32_t* e) {
  const uint32_t lane = prim::lane();
  int64_t hi = t;  // tiles [hi - 64, hi) are read next
  for (uint32_t polls = 0;;) {
    const int64_t j = hi - 1 - (int64_t)lane;  // lane 0 newest
    uint64_t d = 0;
    if (j >= 0) d = prim::ld_agent(a.desc + j);
    const bool ok = j >= 0 && doc_current(d, epoch);
    const uint64_t Kn = prim::ballot(ok && dd_ek(d));
    const uint64_t Pn = prim::ballot(j >= 0 && !ok);
    const int f = Kn ? __builtin_ctzll(Kn) : 64;
    if (Pn & lanes_below(f + (f < 64 ? 1 : 0))) {
      if (++polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); *e = 0; return false; }
      doc_poll_sleep(polls);
      continue;
    }
    if (Kn) { *e = prim::readlane(dd_eo(d), f); return true; }
    hi -= 64;
    polls = 0;
    if (hi <= 0) { *e = 0; return true; }  // cannot happen: tile 0 always knows it
  }
}

// The class of the byte before tile t from tile t - 1's descriptor.
JSIDX_DEV bool doc_pred_walk(const DocArgs& a, int64_t t, uint32_t epoch, uint32_t* p) {
  for (uint32_t polls = 0;;) {
    uint64_t d = 0;
    if (prim::lane() == 0) d = prim::ld_agent(a.desc + t - 1);
    const uint32_t lo = prim::readlane((uint32_t)d, 0), hi = prim::readlane((uint32_t)(d >> 32), 0);
    d = ((uint64_t)hi << 32) | lo;
    if (doc_current(d, epoch)) { *p = dd_po(d); return true; }
    if (++polls > prim::kSpinLimit) { prim::st_agent32(&a.ws->diag, 1u); *p = 0; return false; }
    doc_poll_sleep(polls);
  }
}

// ---- a tile: local pass and publication ------------------------------------------------
JSIDX_DEV bool doc_interior(const DocArgs& a, int64_t t) {
  return t > 0 && a.p0 + (t + 1) * (int64_t)kDocTile < (int64_t)a.len;  // (t > 0: P0 > 64)
}

// The local pass of tile T (S: its prefetched loads, if interior) and its
// descriptor.  Returns the block counter's value before this tile counted
// itself, in lane 0 (the caller reads it later, so the atomic's round trip
// overlaps other work).
template <int VAR>
JSIDX_DEV uint32_t doc_start_tile(const DocArgs& a, DocWaveShared& sh, DocTile& T, uint32_t epoch, const DocPre& S) {
  const uint32_t lane = prim::lane();
  const int64_t t = T.t;
  prim::dtrace(t, 0);
  const bool interior = doc_interior(a, t);
  Behind B;
  B.e = 0; B.p = 1; B.e_known = 1; B.p_known = 1; B.uc = u8_carry_zero();
  if (interior) {
    doc_local_fast<VAR, false>(a, sh, T, &B, true, S);
    if (!B.p_known) {
      // a quote right before the tile after 63 or more backslashes: its
      // class comes from the tile before (rare; the pass is redone)
      doc_pred_walk(a, t, epoch, &B.p);
      B.p_known = 1;
      DocPre S2;
      doc_prefetch(a, T.P0, S2);
      doc_local_fast<VAR, true>(a, sh, T, &B, !B.e_known, S2);
    }
  } else {
    if (t > 0) {
      B = read_behind(a, T.P0);
      if (!B.p_known) doc_pred_walk(a, t, epoch, &B.p);
    }
    doc_local<VAR>(a, sh, T, B.e, B.p, B.uc, !B.e_known);
  }
  T.ek = 1;
  if (!B.e_known) {
    // 64 or more backslashes before the tile: the tile's result depends on
    // the escape entering it only if its first non-backslash byte is a quote,
    // or if the document ends inside the leading run (its trailing flag)
    const bool dep = T.lead_q || T.P0 + (int64_t)T.lead_pos >= (int64_t)a.len;
    if (dep) {
      uint32_t e = 0;
      doc_escape_walk(a, t, epoch, &e);
      if (e) {
        B.e = 1;
        if (interior) {
          DocPre S2;
          doc_prefetch(a, T.P0, S2);
          doc_local_fast<VAR, true>(a, sh, T, &B, false, S2);
        } else {
          doc_local<VAR>(a, sh, T, 1u, B.p, B.uc, false);
        }
      }
    } else if (T.lead_pos >= (uint32_t)kDocTile) {
      T.ek = 0;  // all backslashes: the escape passes through unchanged
    }
  }
  prim::dtrace(t, 1);
  const uint64_t side = doc_side(T.u, T.ek, T.eo, T.po);
  if (lane == 0) {
    if (t == 0) prim::st_agent(a.desc + t, doc_inc(T.qpar, T.c0, side, epoch));
    else prim::st_agent(a.desc + t, doc_agg(T.qpar, T.c0, T.c1, side, epoch));
  }
  // count the block's published tiles (the last one folds the block; it polls
  // until every descriptor of the block is visible, so the count need not
  // wait for the store)
  uint32_t old = 0;
  if (lane == 0) old = prim::add_agent32(a.bcnt + t / kDocBlock, 1u);
  return old;
}

// After the block counter's value is known: the last tile of a block to
// publish folds it.
JSIDX_DEV void doc_after_count(const DocArgs& a, int64_t t, uint32_t oldv, uint32_t epoch) {
  const uint32_t old = prim::readlane(oldv, 0);
  const int64_t b = t / kDocBlock;
  const int64_t nb = a.ntiles - b * kDocBlock < kDocBlock ? a.ntiles - b * kDocBlock : kDocBlock;
  if ((int64_t)old == nb - 1) {
    prim::dcount(t, 1ull << 24);
    doc_fold_block(a, b, epoch, t);
  }
  prim::dtrace(t, 2);
}

// Positions of F (this lane's 32 bytes start at document position rel) at
// ranks from *cc plus the lanes below; *cc advances by the row's count.
// Rows are staged in alternate halves of the buffer, so that a row's writes
// never meet the previous row's reads (the wave waits for its LDS accesses
// once per staged row, which also covers the reads of the row before).
template <bool STAGED>
JSIDX_DEV void doc_write_row(uint32_t* out, uint32_t* stage, uint32_t* half, uint32_t* cc, uint32_t F, uint32_t rel,
                             uint64_t lim) {
  const uint32_t n = (uint32_t)__builtin_popcount(F);
  const uint32_t incl = prim::incl_scan(n);
  const uint32_t row_n = prim::readlane(incl, 63);
  if (row_n == 0) return;
  const uint32_t base = *cc;
  *cc += row_n;
  const bool safe = (uint64_t)base + row_n <= lim;
  if (STAGED && safe && row_n <= (uint32_t)(kDocStage / 2) &&
      prim::ballot(n > (uint32_t)JSIDX_DOC_STAGE_LANE) != 0ull) {
    uint32_t* sb = stage + *half;
    *half ^= (uint32_t)(kDocStage / 2);
    uint32_t k = incl - n;
    while (F) {
      const uint32_t j = (uint32_t)__builtin_ctz(F);
      F &= F - 1u;
      sb[k++] = rel + j;
    }
    prim::wave_sync();
    // four positions per lane and store, then the last few one by one
    const uint32_t full = row_n & ~3u;
    for (uint32_t i = 4u * prim::lane(); i < full; i += 4u * (uint32_t)kThreads)
      prim::st_out4(out + base + i, prim::ld_lds128(sb + i));
    const uint32_t i = full + prim::lane();
    if (i < row_n) prim::st_out(out + base + i, sb[i]);
    return;
  }
  uint32_t k = base + incl - n;
  if (safe) {
    while (F) {
      const uint32_t j = (uint32_t)__builtin_ctz(F);
      F &= F - 1u;
      prim::st_out(out + k, rel + j);
      k++;
    }
  } else {
    while (F) {
      const uint32_t j = (uint32_t)__builtin_ctz(F);
      F &= F - 1u;
      if ((uint64_t)k < lim) prim::st_out(out + k, rel + j);
      k++;
    }
  }
}

// ---- a tile: look-back and finish pass ---------------------------------------------------
// The wave's next tile from its workgroup's pool; the wave that finds the
// batch used up claims the next batch from the global counter (batches, and
// tiles inside a batch, go out in increasing order, only to running waves).
JSIDX_DEV uint32_t doc_take(const DocArgs& a) {
  DocGroupShared& gs = prim::lds_object<DocGroupShared>();
  uint32_t tile = 0;
  if (prim::lane() == 0) {
    for (;;) {
      const uint32_t old = prim::add_lds32(&gs.pool, 1u);
      const uint32_t g = old >> 8, taken = old & 0xFFu;
      if (taken < kDocBatch) { tile = g * kDocBatch + taken; break; }
      if (taken == kDocBatch) {
        const uint32_t ng = prim::add_agent32(&a.ws->ticket, 1u);
        prim::st_lds32(&gs.pool, (ng << 8) | 1u);
        tile = ng * kDocBatch;
        break;
      }
      while ((prim::ld_lds32(&gs.pool) >> 8) == g) prim::sleep();  // another wave claims the next batch
    }
  }
  return prim::readlane(tile, 0);
}

// The wave's next tile, and its first loads if it is interior.
JSIDX_DEV uint32_t doc_next_tile(const DocArgs& a, DocPre* S) {
  const uint32_t nx = doc_take(a);
  if ((int64_t)nx < a.ntiles && doc_interior(a, (int64_t)nx)) doc_prefetch(a, a.p0 + (int64_t)nx * kDocTile, *S);
  return nx;
}

// Tile T's look-back; then the block fold of tile fold_t if it was the last
// of its block to count itself (fold_cnt: the count's old value; fold_t < 0:
// none), so that the fold waits for no flatten; then (once this wave no
// longer waits for anything) its next ticket and first loads into *nx / *S,
// then T's positions.
template <int VAR>
JSIDX_DEV void doc_finish_tile(const DocArgs& a, DocWaveShared& sh, const DocTile& T, uint32_t epoch, uint32_t* nx,
                               DocPre* pre, const LbPre* lb, int64_t fold_t = -1, uint32_t fold_cnt = 0) {
  const uint32_t lane = prim::lane();
  const int64_t t = T.t;
  DocFold S0;
  S0.known = 1; S0.q = 0; S0.u = 0; S0.c0 = 0; S0.c1 = 0; S0.pending = 0;
  prim::dtrace(t, 3);
  if (t > 0) {
    if (!doc_look_back(a, t, epoch, &S0, lb)) { S0.q = 0; S0.u = 0; S0.c0 = 0; }
    // the tile's inclusive value shortens later look-backs in its block
    if (lane == 0) {
      const uint32_t cnt = S0.c0 + (S0.q ? T.c1 : T.c0);
      prim::st_agent(a.desc + t, doc_inc(S0.q ^ T.qpar, cnt, doc_side(S0.u | T.u, T.ek, T.eo, T.po), epoch));
    }
  }
  prim::dtrace(t, 4);
  if (fold_t >= 0) doc_after_count(a, fold_t, fold_cnt, epoch);
  if (nx) *nx = doc_next_tile(a, pre);
  const DocFold& S = S0;
  // the rows' index masks, all loaded before the first write; the slot is
  // then free for staging
  uint2(*m)[kThreads] = sh.m[T.slot];
  uint32_t Fr[kDocRows];
#pragma unroll
  for (int r = 0; r < kDocRows; r++) {
    const uint2 kf = m[r][lane];
    Fr[r] = S.q ? (kf.y ^ kf.x) : kf.y;
  }
  prim::wave_sync();
  uint32_t* stage = reinterpret_cast<uint32_t*>(&m[0][0]);
  uint32_t cc = S.c0;
  uint32_t half = 0;
  const uint64_t lim = a.len;
#pragma unroll
  for (int r = 0; r < kDocRows; r++) {
    const int64_t rel = T.P0 + (int64_t)r * kRowBytes + (int64_t)lane * kSegBytes;
    doc_write_row<(VAR & kVarDirectFlatten) == 0>(a.out_idx, stage, &half, &cc, Fr[r], (uint32_t)rel, lim);
  }
  if (t == a.ntiles - 1 && lane == 0) {
    const uint32_t q = S.q ^ T.qpar, u = S.u | T.u;
    uint32_t err = 0;
    if (u) err |= JSIDX_ERR_UTF8;
    if (q) err |= JSIDX_ERR_UNCLOSED_STRING;
    if (T.tesc) err |= JSIDX_ERR_TRAILING_ESCAPE;
    if (cc == 0) err |= JSIDX_ERR_EMPTY;
    prim::st_out(a.out_n, cc);
    prim::st_out(a.out_err, err);
  }
  prim::wave_sync();
  prim::dtrace(t, 5);
}

// ---- the launch ------------------------------------------------------------------------
template <int VAR = 0>
JSIDX_DEV void doc_tiles(const DocArgs& a) {
  DocGroupShared& gs = prim::lds_object<DocGroupShared>();
  const uint32_t wv = prim::wave_id();
  DocWaveShared& sh = gs.w[wv];
  const uint32_t lane = prim::lane();
  Workspace* ws = a.ws;
  uint32_t epoch = 0;
  if (lane == 0) epoch = prim::ld_agent32(&ws->epoch);
  epoch = prim::readlane(epoch, 0);

  if ((uint64_t)a.ntiles > a.cap) {
    if (prim::block() == 0 && wv == 0 && lane == 0) {
      prim::st_out(a.out_n, 0u);
      prim::st_out(a.out_err, JSIDX_ERR_CAPACITY);
    }
  } else {
    // A workgroup takes its waves' first tiles with one atomic, then each
    // wave takes one tile at a time: tiles go only to running waves, in
    // increasing order.  A wave starts its next tile before finishing the
    // current one; every tile publishes before its wave waits for anything.
    if (wv == 0 && lane == 0) gs.pool = prim::add_agent32(&ws->ticket, 1u) << 8;
    prim::sync();
    uint32_t tk = doc_take(a);
    DocTile pq[kDocSlots - 1];  // published tiles waiting for their finish pass, oldest first
    int np = 0;
    uint32_t slot = 0;
    DocPre S;
    if ((int64_t)tk < a.ntiles && doc_interior(a, (int64_t)tk)) doc_prefetch(a, a.p0 + (int64_t)tk * kDocTile, S);
    while ((int64_t)tk < a.ntiles) {
      DocTile T;
      T.t = (int64_t)tk;
      T.P0 = a.p0 + T.t * (int64_t)kDocTile;
      T.slot = slot;
      // the look-back reads of the tile finished after this local pass go out now
      LbPre lb;
      if (np == kDocSlots - 1) doc_lb_issue(a, pq[0].t, lb);
      const uint32_t cnt = doc_start_tile<VAR>(a, sh, T, epoch, S);
      uint32_t nx = 0;
      if (np == kDocSlots - 1) {
        doc_finish_tile<VAR>(a, sh, pq[0], epoch, &nx, &S, &lb, T.t, cnt);
#pragma unroll
        for (int i = 0; i + 1 < kDocSlots - 1; i++) pq[i] = pq[i + 1];
        np--;
      } else {
        nx = doc_next_tile(a, &S);
        doc_after_count(a, T.t, cnt, epoch);
      }
#pragma unroll
      for (int i = 0; i < kDocSlots - 1; i++)
        if (i == np) pq[i] = T;
      np++;
      slot = slot + 1u == (uint32_t)kDocSlots ? 0u : slot + 1u;
      tk = nx;
    }
#pragma unroll
    for (int i = 0; i < kDocSlots - 1; i++)
      if (i < np) doc_finish_tile<VAR>(a, sh, pq[i], epoch, nullptr, nullptr, nullptr);
  }

  // The last workgroup out resets the counters for the next launch, clears
  // the block words and a rotating window of tile descriptors (so that no
  // stale descriptor can ever carry a matching epoch), and writes the result
  // of an empty document.
  prim::sync();
  if (wv == 0 && lane == 0) {
    prim::wait_mem();
    const uint32_t old = prim::add_agent32(&ws->done, 1u);
    gs.is_last = (old == prim::grid() - 1) ? 1u : 0u;
  }
  prim::sync();
  if (gs.is_last) {
    const uint64_t gl = (uint64_t)wv * kThreads + lane;
    const uint64_t nwin = (a.cap + kDocScrub - 1) / kDocScrub;
    const uint64_t w0 = (uint64_t)(epoch % (uint32_t)(nwin ? nwin : 1)) * kDocScrub;
    for (uint64_t j = w0 + gl; j < w0 + kDocScrub && j < a.cap; j += kDocThreads) prim::st_agent(a.desc + j, 0ull);
    const uint64_t nb = doc_blocks_for((uint64_t)(a.ntiles > 0 ? a.ntiles : 0));
    for (uint64_t j = gl; j < nb; j += kDocThreads) {
      prim::st_agent(a.blk + 2 * j, 0ull);
      prim::st_agent(a.blk + 2 * j + 1, 0ull);
      prim::st_agent32(a.bcnt + j, 0u);
    }
    if (a.ntiles == 0 && gl == 0) {
      prim::st_out(a.out_n, 0u);
      prim::st_out(a.out_err, JSIDX_ERR_EMPTY);
    }
    prim::sync();
    if (wv == 0 && lane == 0) {
      prim::st_agent32(&ws->ticket, 0u);
      prim::st_agent32(&ws->done, 0u);
      prim::st_agent32(&ws->epoch, epoch + 1u);
    }
  }
}

}  // namespace jsidx
