// jsidx_kernel.h -- the stage-1 indexing kernel body (see jsidx.hip for the
// design summary).  Written against the primitives of jsidx_prims.h only.
#pragma once
#include <stdint.h>

#include "jsidx.h"
#include "jsidx_device.h"

namespace jsidx {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kSegBytes = 32;
constexpr int kRowBytes = kThreads * kSegBytes;  // 8 KiB
constexpr int kRows = 2;
constexpr int kTileBytes = kRows * kRowBytes;  // 16 KiB
constexpr int kDocCap = 1024;                  // documents per tile held in LDS
constexpr int kScrub = 4096;                   // descriptors cleared per launch

// ---- tile descriptors for the look-back -----------------------------------
// bits 0..2 flag, 3..10 payload, 11..42 count, 43..63 launch epoch (21 bits).
enum : uint32_t { kNone = 0, kStateAgg = 1, kStateInc = 2, kCountAgg = 3, kCountInc = 4 };
constexpr uint32_t kEpochBits = 21;
constexpr uint32_t kEpochMask = (1u << kEpochBits) - 1u;

struct Workspace {
  uint32_t ticket;  // next tile to hand out
  uint32_t done;    // workgroups that have left the tile loop
  uint32_t epoch;   // launch counter (tags descriptors)
  uint32_t diag;    // sticky: 1 = a look-back wait gave up (never expected)
  uint64_t desc[1];  // one per tile
};

JSIDX_DEV uint64_t make_desc(uint32_t flag, uint32_t payload, uint32_t count, uint32_t epoch) {
  return (uint64_t)flag | ((uint64_t)(payload & 0xFFu) << 3) | ((uint64_t)count << 11) |
         ((uint64_t)(epoch & kEpochMask) << 43);
}
JSIDX_DEV uint32_t desc_flag(uint64_t d) { return (uint32_t)(d & 7u); }
JSIDX_DEV uint32_t desc_payload(uint64_t d) { return (uint32_t)((d >> 3) & 0xFFu); }
JSIDX_DEV uint32_t desc_count(uint64_t d) { return (uint32_t)(d >> 11); }
JSIDX_DEV uint32_t desc_epoch(uint64_t d) { return (uint32_t)(d >> 43); }

JSIDX_DEV uint64_t ld_desc(Workspace* ws, int64_t j) {
  return prim::ld_agent(&ws->desc[j]);
}
JSIDX_DEV void st_desc(Workspace* ws, int64_t j, uint64_t v) {
  prim::st_agent(&ws->desc[j], v);
}

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
// A then B.
JSIDX_DEV uint32_t tab_compose(uint32_t A, uint32_t B) {
  uint32_t C = (A & 1u) | (B & 1u);
  uint32_t bu = (B >> 1) & 1u;
  uint32_t cu = (B & 1u) ? bu : (((A >> 1) & 1u) | bu);
  C |= cu << 1;
#pragma unroll
  for (uint32_t e = 0; e < 2; e++) {
    uint32_t a = (A >> (2 + 3 * e)) & 7u;
    uint32_t b = (B >> (2 + 3 * (a & 1u))) & 7u;
    uint32_t q = (B & 1u) ? ((b >> 1) & 1u) : (((a >> 1) ^ (b >> 1)) & 1u);
    uint32_t ent = (b & 1u) | (q << 1) | (b & 4u);
    C |= ent << (2 + 3 * e);
  }
  return C;
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
  uint64_t cap_tiles;  // descriptors available
};

JSIDX_DEV int64_t doc_off(const Args& a, int64_t d) {
  if (a.offsets) return (int64_t)prim::load8(a.offsets + d);
  return d <= 0 ? 0 : (int64_t)a.len;
}

// ---- per-lane, per-row state ----------------------------------------------
struct Seg {
  uint32_t C, W, Q, R, PR, EA;  // classes, in-string, predecessor, escape-after
  uint32_t Qraw, B;
  uint32_t D;    // document starts at bits 0..31
  uint32_t d32;  // a document starts right after bit 31
  uint32_t V;    // bytes inside [begin, end)
  uint32_t UE;   // UTF-8 error of the piece starting at this bit
  int32_t head;  // local index of the document holding bit 0 (-1: none)
  uint32_t F;    // final index bits
  uint32_t cin;  // output rank of the first head bit
  uint32_t uin;  // UTF-8 error of the head document before this segment
};

struct Shared {
  int64_t tile;
  int64_t d_first;
  int64_t first_off;
  int32_t ntab;
  int32_t overflow;
  int32_t tab[kDocCap + 1];
  // wave aggregates, [row][wave]
  uint32_t agg_a[kRows][kWaves];
  uint32_t agg_b[kRows][kWaves];
  uint32_t agg_c[kRows][kWaves];
  // tile facts
  uint32_t lead_pos;  // first byte that is not a backslash or starts a doc
  uint32_t qsens;     // that byte is a quote (its escape depends on e_in)
  uint32_t r0;        // first document start in the tile (kTileBytes: none)
  uint32_t state_in;  // carry-in state
  uint32_t base;      // rank of the tile's first head bit
  uint32_t is_last;
  uint32_t epoch;
  int32_t min_reset;
};

// Local document index of tile-relative position rel: the last document
// starting at or before it (empty documents at the same place come first).
// (Only used while the table holds every document of the tile.)
JSIDX_DEVFN int32_t local_doc_of(const Shared& sh, int32_t rel) {
  int32_t lo = 0, hi = sh.ntab;  // first entry > rel
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

JSIDX_DEV uint32_t lane_id() { return prim::lane(); }
JSIDX_DEV uint64_t lt_lanes() {
  uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}
JSIDX_DEV int msb64(uint64_t m) { return 63 - __builtin_clzll(m); }

// Mask bytes of word k (bytes 4k..4k+3 of the segment) by the bit mask keep.
JSIDX_DEV uint32_t keep_bytes(uint32_t w, uint32_t keep, int k) {
  return w & nibble_bytemask((keep >> (4 * k)) & 0xFu);
}

// UTF-8 errors of the bytes kept by `keep` (others read as 0x00), with the
// word before the segment `halo` and, if tail, a zero word after it.
JSIDX_DEVFN uint32_t utf8_piece(const uint32_t w[8], uint32_t halo, uint32_t keep, bool tail) {
  Utf8Word prev = utf8_lookup_raw(halo);
  uint32_t err = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) {
    uint32_t x = keep_bytes(w[k], keep, k);
    Utf8Word cur = utf8_lookup_raw(x);
    err |= utf8_pair_errors(prev, cur);
    prev = cur;
  }
  if (tail) err |= utf8_pair_errors(prev, utf8_lookup_raw(0u));
  return err;
}

// ---------------------------------------------------------------------------
JSIDX_DEVFN void index_tiles(const Args& a) {
  Shared& sh = prim::lds_object<Shared>();
  const uint32_t tid = prim::tid();
  const uint32_t wave = tid >> 6;
  const uint32_t lane = tid & 63u;
  Workspace* ws = a.ws;

  if (tid == 0) sh.epoch = prim::ld_agent32(&ws->epoch);
  prim::sync();
  const uint32_t epoch = sh.epoch;

  const int64_t begin = doc_off(a, 0);
  const int64_t end = doc_off(a, (int64_t)a.ndocs);
  const uintptr_t base_addr = (uintptr_t)a.base;
  const uintptr_t g0 = (base_addr + (uintptr_t)begin) & ~(uintptr_t)15;
  const int64_t pos_g0 = (int64_t)(g0 - base_addr);  // position of tile 0 byte 0
  int64_t span = end - pos_g0;
  int64_t ntiles = span > 0 ? (span + kTileBytes - 1) / kTileBytes : 1;

  if ((uint64_t)ntiles > a.cap_tiles) {
    // Not indexed: flag every document.
    for (int64_t d = (int64_t)prim::block() * kThreads + tid; d < a.ndocs; d += (int64_t)prim::grid() * kThreads) {
      prim::st_out(a.out_n + d, 0u);
      prim::st_out(a.out_err + d, JSIDX_ERR_CAPACITY);
    }
    goto finish;
  }

  while (true) {
    if (tid == 0) sh.tile = (int64_t)prim::add_agent32(&ws->ticket, 1u);
    prim::sync();
    const int64_t t = sh.tile;
    if (t >= ntiles) break;
    prim::trace(t, 0);
    const int64_t P0 = pos_g0 + t * kTileBytes;  // position of tile byte 0
    const int64_t Pend = P0 + kTileBytes;

    // ---- documents of this tile -------------------------------------------
    // d_first: the first document whose end is at or after the tile start.
    if (wave == 0) {
      int64_t lo = 0, hi = (int64_t)a.ndocs - 1;
      while (lo < hi) {
        int64_t step = (hi - lo + 64) / 64;
        int64_t d = lo + (int64_t)lane * step;
        bool ok = d <= hi;
        bool pr = ok && doc_off(a, d + 1) >= P0;
        uint64_t b = prim::ballot(pr);
        int64_t f = b ? (int64_t)__builtin_ctzll(b) : -1;
        int64_t dfound = f >= 0 ? lo + f * step : hi;
        int64_t nprobe = (hi - lo) / step;  // last valid probe lane
        if (nprobe > 63) nprobe = 63;
        int64_t nlo = f > 0 ? lo + (f - 1) * step + 1 : (f == 0 ? lo : lo + nprobe * step + 1);
        lo = nlo;
        hi = dfound;
      }
      if (lane == 0) {
        sh.d_first = lo;
        sh.first_off = doc_off(a, lo);
        sh.overflow = 0;
        sh.ntab = 0;
        sh.min_reset = 0x7FFFFFFF;
      }
    }
    prim::sync();
    const int64_t d_first = sh.d_first;
    // Table of starts of documents d_first.. with start <= Pend, relative to P0;
    // entry 0 clamped at -1.  Empty documents owned by this tile are finished
    // here: the tile owning a position owns the empty documents there.
    {
      int32_t count = 0;
      for (int64_t i0 = 0;; i0 += kThreads) {
        int64_t d = d_first + i0 + tid;
        bool in = d <= (int64_t)a.ndocs;
        int64_t o = in ? doc_off(a, d) : 0;
        in = in && o <= Pend;
        if (in && i0 + tid < kDocCap + 1) {
          int64_t r = o - P0;
          sh.tab[i0 + tid] = (int32_t)(r < -1 ? -1 : r);
        }
        if (in && d < (int64_t)a.ndocs) {
          int64_t o2 = doc_off(a, d + 1);
          bool owned = (o >= P0 && o < Pend) || (o == end && t == ntiles - 1);
          if (o2 == o && owned) {
            prim::st_out(a.out_n + d, 0u);
            prim::st_out(a.out_err + d, JSIDX_ERR_EMPTY);
          }
        }
        int n_in = prim::sync_count(in);
        count += n_in;
        if (n_in < kThreads) break;
      }
      if (tid == 0) {
        sh.ntab = count;
        sh.overflow = count > kDocCap + 1;
      }
    }
    prim::sync();

    prim::trace(t, 1);
    // ---- phase 1: load, classify, local scans -------------------------------
    Seg sg[kRows];
#pragma unroll
    for (int r = 0; r < kRows; r++) {
      Seg& s = sg[r];
      const int32_t rel = r * kRowBytes + (int32_t)tid * kSegBytes;  // tile-relative
      const int64_t pos = P0 + rel;
      // documents
      int32_t lo;
      if (!sh.overflow) {
        lo = local_doc_of(sh, rel);
      } else {
        lo = (int32_t)(global_upper(a, d_first, (int64_t)a.ndocs + 1, pos) - 1 - d_first);
      }
      s.head = lo;
      uint32_t D = 0, d32 = 0;
      for (int32_t i = lo < 0 ? 0 : lo;; i++) {
        int64_t o;
        if (!sh.overflow) {
          if (i >= sh.ntab) break;
          o = (int64_t)sh.tab[i] + P0;
          if (i == 0) o = sh.first_off;
        } else {
          if (d_first + i > (int64_t)a.ndocs) break;
          o = doc_off(a, d_first + i);
        }
        if (o < pos) continue;
        if (o > pos + 32) break;
        if (o == pos + 32) d32 = 1; else D |= 1u << (uint32_t)(o - pos);
      }
      s.D = D;
      s.d32 = d32;
      int64_t vlo = begin - pos, vhi = end - pos;
      uint32_t V = ge_mask((uint32_t)(vlo < 0 ? 0 : (vlo > 32 ? 32 : vlo))) &
                   lt_mask((uint32_t)(vhi < 0 ? 0 : (vhi > 32 ? 32 : vhi)));
      s.V = V;
      if (s.head >= 0 && d_first + s.head >= (int64_t)a.ndocs) s.head = -1;

      // load the 32 bytes and the 4 bytes before them
      uint32_t w[8];
      const uint8_t* p = a.base + pos;  // 16-byte aligned
      // only granules overlapping [begin, end) are read
#pragma unroll
      for (int h = 0; h < 2; h++) {
        if (begin < end && pos + 16 * h < end && pos + 16 * h + 16 > begin) {
          uint4 v = prim::load16(p + 16 * h);
          w[4 * h + 0] = v.x; w[4 * h + 1] = v.y; w[4 * h + 2] = v.z; w[4 * h + 3] = v.w;
        } else {
          w[4 * h + 0] = w[4 * h + 1] = w[4 * h + 2] = w[4 * h + 3] = 0u;
        }
      }
      // The 4 bytes before the segment, as far as they belong to the document
      // holding byte 0 (UTF-8 context); 0x00 otherwise.
      uint32_t halo = 0;
      if (s.head >= 0 && !(D & 1u) && begin < end && pos > begin && pos - 16 < end) {
        halo = prim::load4(p - 4);
        int64_t hd_off = s.head == 0 ? sh.first_off
                                     : (!sh.overflow ? (int64_t)sh.tab[s.head] + P0 : doc_off(a, d_first + s.head));
        int64_t hlo = hd_off - (pos - 4);  // halo bytes before the document start
        if (hlo > 0) halo &= hlo >= 4 ? 0u : (~0u << (8 * hlo));
      }
      if (V != ~0u) {
#pragma unroll
        for (int k = 0; k < 8; k++) w[k] = keep_bytes(w[k], V, k);
      }

      uint32_t hidx[8], sgn[8];
      ClassMasks cm = classify_segment(w, hidx, sgn);
      s.C = cm.C; s.W = cm.W; s.Qraw = cm.Q; s.B = cm.B;

      // UTF-8 errors, per piece of the segment (pieces start at bit 0 and at
      // every document start).  Waves without non-ASCII bytes skip it.
      s.UE = 0;
      bool need = (cm.hi | (halo & 0x80808080u)) != 0u;
      if (prim::ballot(need) != 0ull) {
        if (D == 0 && !d32) {
          // one piece, continued on both sides
          Utf8Word prev = utf8_lookup_raw(halo);
          uint32_t err = 0;
#pragma unroll
          for (int k = 0; k < 8; k++) {
            Utf8Word cur = utf8_lookup(w[k], hidx[k], sgn[k]);
            err |= utf8_pair_errors(prev, cur);
            prev = cur;
          }
          s.UE = err ? 1u : 0u;
        } else {
          uint32_t starts = D | 1u;
          while (starts) {
            uint32_t st = (uint32_t)__builtin_ctz(starts);
            starts &= starts - 1u;
            uint32_t nx = starts ? (uint32_t)__builtin_ctz(starts) : 32u;
            bool ends_doc = nx < 32u || d32;
            uint32_t keep = ge_mask(st) & lt_mask(nx);
            uint32_t hh = (st == 0 && !(D & 1u)) ? halo : 0u;
            if (utf8_piece(w, hh, keep, ends_doc)) s.UE |= 1u << st;
          }
        }
      }
    }

    prim::trace(t, 2);
    // ---- escape scan -----------------------------------------------------
    // A segment with a non-backslash byte or a document start fixes the escape
    // state after it; an all-backslash segment (32 bytes, even) passes it on.
    uint32_t e_out_c[kRows];
#pragma unroll
    for (int r = 0; r < kRows; r++) {
      Seg& s = sg[r];
      bool isconst = (s.B != ~0u) || (s.D != 0u);
      uint32_t hi_reset = s.D ? 31u - (uint32_t)__builtin_clz(s.D) : 0u;
      uint32_t last_b = s.B & ge_mask(hi_reset);
      uint32_t nb = ~last_b;
      e_out_c[r] = (nb ? (uint32_t)__builtin_clz(nb) : 32u) & 1u;
      uint64_t K = prim::ballot(isconst);
      uint64_t E = prim::ballot(e_out_c[r] != 0u);
      if (lane == 0) sh.agg_a[r][wave] = K ? (1u | ((uint32_t)((E >> msb64(K)) & 1ull) << 1)) : 0u;
    }
    prim::sync();
    // carry-in per (row, wave) with e_T = 0; tile-level facts
    uint32_t e_in[kRows];
    {
      uint32_t e = 0;
      uint32_t any_const = 0;
#pragma unroll
      for (int r = 0; r < kRows; r++) {
        for (int wv = 0; wv < kWaves; wv++) {
          uint32_t ag = sh.agg_a[r][wv];
          if (wv == (int)wave) {
            Seg& s = sg[r];
            bool isconst = (s.B != ~0u) || (s.D != 0u);
            uint64_t K = prim::ballot(isconst);
            uint64_t E = prim::ballot(e_out_c[r] != 0u);
            uint64_t m = K & lt_lanes();
            e_in[r] = m ? (uint32_t)((E >> msb64(m)) & 1ull) : e;
            // the first state-fixing segment of the tile reports its lead byte
            if (!any_const && K && lane == (uint32_t)__builtin_ctzll(K)) {
              uint32_t p = (uint32_t)__builtin_ctz(~s.B | s.D);
              bool reset_first = (s.D >> p) & 1u;
              sh.lead_pos = (uint32_t)(r * kRowBytes) + tid * kSegBytes + p;
              sh.qsens = reset_first ? 0u : ((s.Qraw >> p) & 1u);
            }
          }
          if (ag & 1u) { e = (ag >> 1) & 1u; any_const = 1; }
        }
      }
      if (tid == 0 && !any_const) { sh.lead_pos = kTileBytes; sh.qsens = 0; }
      if (tid == 0) sh.agg_c[0][0] = any_const | (e << 1);
    }
    prim::sync();
    const uint32_t tile_any_const = sh.agg_c[0][0] & 1u;
    const uint32_t tile_e_last = (sh.agg_c[0][0] >> 1) & 1u;

    // ---- escapes, quotes, string ranges, predecessor bits ------------------
    uint32_t qval[kRows], pbit[kRows], uval[kRows];
#pragma unroll
    for (int r = 0; r < kRows; r++) {
      Seg& s = sg[r];
      uint32_t OD = escaped_bytes(s.B, s.D, e_in[r], &s.EA);
      s.Q = s.Qraw & ~OD;
      uint32_t PX = prefix_xor(s.Q);
      uint32_t corr = 0, c_old = 0, rest = s.D;
      while (rest) {
        uint32_t d = (uint32_t)__builtin_ctz(rest);
        rest &= rest - 1u;
        uint32_t c_new = d ? ((PX >> (d - 1u)) & 1u) : 0u;
        if (c_new != c_old) corr ^= ge_mask(d);
        c_old = c_new;
      }
      s.R = PX ^ corr;  // with q_in = 0
      qval[r] = s.D ? (s.R >> 31) : (uint32_t)(__builtin_popcount(s.Q) & 1);
      uint32_t P0m = s.C | s.W | s.Q;
      s.PR = P0m << 1;  // bit 0 filled after the scan
      pbit[r] = P0m >> 31;
      // UTF-8: value passed on: the last piece's error (reset) or the segment's
      uint32_t last_start = s.D ? 31u - (uint32_t)__builtin_clz(s.D) : 0u;
      uval[r] = (s.UE >> last_start) & 1u;
      if (!s.D) uval[r] = s.UE & 1u;
      uint64_t Rs = prim::ballot(s.D != 0u);
      uint64_t Qv = prim::ballot(qval[r] != 0u);
      uint64_t Uv = prim::ballot(uval[r] != 0u);
      uint64_t Pb = prim::ballot(pbit[r] != 0u);
      if (lane == 0) {
        uint64_t from = Rs ? (~0ull << msb64(Rs)) : ~0ull;
        uint32_t qp = (uint32_t)(__builtin_popcountll(Qv & from) & 1);
        uint32_t uo = (Uv & from) ? 1u : 0u;
        sh.agg_a[r][wave] = (Rs ? 1u : 0u) | (qp << 1) | (uo << 2) | ((uint32_t)(Pb >> 63) << 3);
      }
      if (Rs && lane == (uint32_t)__builtin_ctzll(Rs)) {
        int32_t rp = r * kRowBytes + (int32_t)tid * kSegBytes + __builtin_ctz(s.D);
        prim::min_lds(&sh.min_reset, rp);
      }
    }
    prim::sync();
    uint32_t tile_state_out;  // with zero carry-in
    uint32_t tile_reset;
    {
      uint32_t q = 0, u = 0, p = 0, any_reset = 0;
#pragma unroll
      for (int r = 0; r < kRows; r++) {
        for (int wv = 0; wv < kWaves; wv++) {
          uint32_t ag = sh.agg_a[r][wv];
          if (wv == (int)wave) {
            Seg& s = sg[r];
            uint64_t Rs = prim::ballot(s.D != 0u);
            uint64_t Qv = prim::ballot(qval[r] != 0u);
            uint64_t Uv = prim::ballot(uval[r] != 0u);
            uint64_t Pb = prim::ballot(pbit[r] != 0u);
            uint64_t m = Rs & lt_lanes();
            uint64_t span_m = m ? (lt_lanes() & ~(msb64(m) ? (~0ull >> (64 - msb64(m))) : 0ull)) : lt_lanes();
            uint32_t qin = (uint32_t)(__builtin_popcountll(Qv & span_m) & 1);
            uint32_t uin = (Uv & span_m) ? 1u : 0u;
            if (!m) { qin ^= q; uin |= u; }
            uint32_t pin = lane ? (uint32_t)((Pb >> (lane - 1)) & 1ull) : p;
            uint32_t first_reset = s.D ? (uint32_t)__builtin_ctz(s.D) : 32u;
            if (qin) s.R ^= lt_mask(first_reset);
            s.PR |= pin;
            s.PR |= s.D;
            s.uin = uin;
          }
          if (ag & 1u) { q = (ag >> 1) & 1u; u = (ag >> 2) & 1u; any_reset = 1; }
          else { q ^= (ag >> 1) & 1u; u |= (ag >> 2) & 1u; }
          p = (ag >> 3) & 1u;
        }
      }
      tile_reset = any_reset;
      tile_state_out = tile_e_last | (q << 1) | (p << 2) | (u << 3);
    }
    // tile transfer table
    const uint32_t lead_pos = sh.lead_pos;
    const uint32_t qsens = sh.qsens;
    const uint32_t r0 = sh.min_reset == 0x7FFFFFFF ? (uint32_t)kTileBytes : (uint32_t)sh.min_reset;
    uint32_t table;
    {
      uint32_t q0 = (tile_state_out >> 1) & 1u, p0 = (tile_state_out >> 2) & 1u, u0 = (tile_state_out >> 3) & 1u;
      table = tile_reset | (u0 << 1);
#pragma unroll
      for (uint32_t e = 0; e < 2; e++) {
        uint32_t eo = tile_any_const ? tile_e_last : e;
        uint32_t flip = e & qsens;
        uint32_t qo = tile_reset ? q0 : (q0 ^ flip);
        uint32_t po = p0 ^ (flip & (lead_pos == (uint32_t)kTileBytes - 1u ? 1u : 0u));
        table |= (eo | (qo << 1) | (po << 2)) << (2 + 3 * e);
      }
    }

    prim::trace(t, 3);
    // ---- phase 2: carry-in state by look-back --------------------------------
    if (wave == 0) {
      uint32_t s_in = 0;
      if (t == 0) {
        if (lane == 0) st_desc(ws, t, make_desc(kStateInc, tab_apply(table, 0u) | (tile_reset << 4), 0, epoch));
      } else {
        if (lane == 0) st_desc(ws, t, make_desc(kStateAgg, table, 0, epoch));
        uint32_t acc = 0;
        bool has_acc = false;
        int64_t jhi = t - 1;
        while (true) {
          int64_t j = jhi - (int64_t)lane;
          uint64_t d = 0;
          if (j >= 0) {
            for (uint32_t spins = 0;; spins++) {
              d = ld_desc(ws, j);
              if (desc_epoch(d) == (epoch & kEpochMask) && desc_flag(d) >= kStateAgg) break;
              if (spins > prim::kSpinLimit) {  // never expected: give up, flag it
                prim::st_agent32(&ws->diag, 1u);
                d = make_desc(kCountInc, 0u, 0u, epoch);
                break;
              }
              prim::sleep();
            }
          }
          uint64_t inc = prim::ballot(j >= 0 && desc_flag(d) >= kStateInc);
          int lim = inc ? __builtin_ctzll(inc) : (int)((jhi + 1) < 64 ? (jhi + 1) : 64);
          uint32_t pay = desc_payload(d);
          // compose the aggregates of lanes lim-1 .. 0 (oldest first)
          uint32_t comp = 0;
          bool has = false;
          for (int i = lim - 1; i >= 0; i--) {
            uint32_t ti = prim::shfl(pay, i);
            comp = has ? tab_compose(comp, ti) : ti;
            has = true;
          }
          if (has) {
            acc = has_acc ? tab_compose(comp, acc) : comp;
            has_acc = true;
          }
          prim::trace_count(t, 8);
          if (inc) {
            uint32_t st = prim::shfl(pay, lim) & 0xFu;
            s_in = has_acc ? tab_apply(acc, st) : st;
            break;
          }
          jhi -= 64;
        }
        if (lane == 0) st_desc(ws, t, make_desc(kStateInc, tab_apply(table, s_in) | (tile_reset << 4), 0, epoch));
      }
      if (lane == 0) sh.state_in = s_in;
    }
    prim::sync();
    prim::trace(t, 4);
    const uint32_t s_in = sh.state_in;
    const uint32_t eT = s_in & 1u, qT = (s_in >> 1) & 1u, pT = (s_in >> 2) & 1u, uT = (s_in >> 3) & 1u;

    // ---- phase 3: apply the carry-in, final masks, counts --------------------
    const uint32_t flipQ = eT & qsens;
    uint32_t cval[kRows];
#pragma unroll
    for (int r = 0; r < kRows; r++) {
      Seg& s = sg[r];
      const uint32_t rel = (uint32_t)(r * kRowBytes) + tid * kSegBytes;
      // head region: tile positions < r0
      uint32_t head = rel >= r0 ? 0u : (r0 - rel >= 32u ? ~0u : lt_mask(r0 - rel));
      uint32_t x = qT ? head : 0u;
      if (flipQ) {
        uint32_t ge = lead_pos <= rel ? ~0u : (lead_pos - rel >= 32u ? 0u : ge_mask(lead_pos - rel));
        x ^= head & ge;
        if (lead_pos >= rel && lead_pos < rel + 32u) s.Q ^= 1u << (lead_pos - rel);
        // the byte after the flipped quote sees a different predecessor
        uint32_t nxt = lead_pos + 1u;
        if (nxt >= rel && nxt < rel + 32u && !((s.D >> (nxt - rel)) & 1u)) s.PR ^= 1u << (nxt - rel);
      }
      s.R ^= x;
      if (rel == 0 && pT) s.PR |= 1u;
      if (eT) {
        // escape state after each byte of the tile's leading backslash run flips
        uint32_t lead = lead_pos <= rel ? 0u : (lead_pos - rel >= 32u ? ~0u : lt_mask(lead_pos - rel));
        s.EA ^= lead & head;
      }
      if (rel < r0) s.uin |= uT;
      uint32_t cwq = s.C | s.W | s.Q;
      s.F = ((s.C & ~s.R) | (s.Q & s.R) | (s.PR & ~s.R & ~cwq)) & s.V;
      uint32_t last_start = s.D ? 31u - (uint32_t)__builtin_clz(s.D) : 0u;
      cval[r] = (uint32_t)__builtin_popcount(s.F & ge_mask(last_start));
      // wave-level segmented scan of counts
      uint32_t S = cval[r];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = prim::shfl_up(S, o);
        if (lane >= (uint32_t)o) S += y;
      }
      uint64_t Rs = prim::ballot(s.D != 0u);
      uint64_t m = Rs & lt_lanes();
      uint32_t Sprev = prim::shfl_up(S, 1);
      if (lane == 0) Sprev = 0;
      int k = m ? msb64(m) : -1;
      uint32_t Sk = prim::shfl(S, k > 0 ? k - 1 : 0);
      if (k <= 0) Sk = 0;
      s.cin = Sprev - Sk;  // lanes [k, lane) (or [0, lane))
      uint32_t tot = prim::shfl(S, 63);
      int kl = Rs ? msb64(Rs) : -1;
      uint32_t Skl = prim::shfl(S, kl > 0 ? kl - 1 : 0);
      if (kl <= 0) Skl = 0;
      if (lane == 0) {
        sh.agg_b[r][wave] = Rs ? 1u : 0u;
        sh.agg_c[r][wave] = tot - Skl;
      }
      // remember whether this lane's carry comes from earlier waves
      s.d32 |= (m ? 0u : 2u);
    }
    prim::sync();
    uint32_t tile_count;
    {
      uint32_t c = 0;
#pragma unroll
      for (int r = 0; r < kRows; r++) {
        for (int wv = 0; wv < kWaves; wv++) {
          if (wv == (int)wave) {
            Seg& s = sg[r];
            if (s.d32 & 2u) s.cin += c;
            s.d32 &= 1u;
          }
          if (sh.agg_b[r][wv]) c = sh.agg_c[r][wv]; else c += sh.agg_c[r][wv];
        }
      }
      tile_count = c;
    }

    prim::trace(t, 5);
    // ---- phase 4: output base by look-back ------------------------------------
    if (wave == 0) {
      uint32_t base = 0;
      uint32_t st_inc = tab_apply(table, s_in) | (tile_reset << 4);
      if (t == 0) {
        if (lane == 0) st_desc(ws, t, make_desc(kCountInc, st_inc, tile_count, epoch));
      } else {
        if (lane == 0) st_desc(ws, t, make_desc(kCountAgg, st_inc, tile_count, epoch));
        int64_t jhi = t - 1;
        while (true) {
          int64_t j = jhi - (int64_t)lane;
          uint64_t d = 0;
          if (j >= 0) {
            for (uint32_t spins = 0;; spins++) {
              d = ld_desc(ws, j);
              if (desc_epoch(d) == (epoch & kEpochMask) && desc_flag(d) >= kCountAgg) break;
              if (spins > prim::kSpinLimit) {  // never expected: give up, flag it
                prim::st_agent32(&ws->diag, 1u);
                d = make_desc(kCountInc, 0u, 0u, epoch);
                break;
              }
              prim::sleep();
            }
          }
          bool stop_l = j >= 0 && (desc_flag(d) == kCountInc || ((desc_payload(d) >> 4) & 1u));
          uint64_t stop = prim::ballot(stop_l);
          int lim = stop ? __builtin_ctzll(stop) : 64;
          uint32_t v = (j >= 0 && (int)lane <= lim) ? desc_count(d) : 0u;
#pragma unroll
          for (int o = 32; o >= 1; o >>= 1) v += prim::shfl_xor(v, o);
          base += v;
          prim::trace_count(t, 9);
          if (stop || jhi < 64) break;
          jhi -= 64;
        }
        if (lane == 0) {
          uint32_t inc = tile_reset ? tile_count : base + tile_count;
          st_desc(ws, t, make_desc(kCountInc, st_inc, inc, epoch));
        }
      }
      if (lane == 0) sh.base = base;
    }
    prim::sync();
    prim::trace(t, 6);
    const uint32_t base = sh.base;

    // ---- phase 5: positions and per-document results ---------------------------
#pragma unroll
    for (int r = 0; r < kRows; r++) {
      Seg& s = sg[r];
      const uint32_t rel = (uint32_t)(r * kRowBytes) + tid * kSegBytes;
      const int64_t pos = P0 + rel;
      if (rel < r0) s.cin += base;
      uint32_t starts = s.D | 1u;
      while (starts) {
        uint32_t st = (uint32_t)__builtin_ctz(starts);
        starts &= starts - 1u;
        uint32_t nx = starts ? (uint32_t)__builtin_ctz(starts) : 32u;
        bool is_head = (st == 0 && !(s.D & 1u));
        int64_t dloc;
        if (is_head) {
          dloc = s.head;
        } else if (!sh.overflow) {
          dloc = local_doc_of(sh, (int32_t)(rel + st));
        } else {
          dloc = global_upper(a, d_first, (int64_t)a.ndocs + 1, pos + st) - 1 - d_first;
        }
        int64_t dglob = d_first + dloc;
        if (dloc < 0 || dglob >= (int64_t)a.ndocs) continue;
        int64_t doff = dloc == 0 ? sh.first_off
                                 : (!sh.overflow ? (int64_t)sh.tab[dloc] + P0 : doc_off(a, dglob));
        uint32_t rank = is_head ? s.cin : 0u;
        uint32_t Fs = s.F & ge_mask(st) & lt_mask(nx);
        uint32_t* out = a.out_idx + doff;
        uint32_t rel_doc = (uint32_t)(pos - doff);
        uint32_t f = Fs;
        uint32_t k = rank;
        while (f) {
          uint32_t j = (uint32_t)__builtin_ctz(f);
          f &= f - 1u;
          if ((uint64_t)(doff + k) < (uint64_t)end) prim::st_out(out + k, rel_doc + j);
          k++;
        }
        bool ends_doc = nx < 32u || s.d32;
        if (ends_doc) {
          uint32_t e = nx - 1u;
          uint32_t n = k;
          uint32_t err = 0;
          uint32_t u8 = ((s.UE >> st) & 1u) | (is_head ? s.uin : 0u);
          if (u8) err |= JSIDX_ERR_UTF8;
          if ((s.R >> e) & 1u) err |= JSIDX_ERR_UNCLOSED_STRING;
          if ((s.EA >> e) & 1u) err |= JSIDX_ERR_TRAILING_ESCAPE;
          if (n == 0) err |= JSIDX_ERR_EMPTY;
          prim::st_out(a.out_n + dglob, n);
          prim::st_out(a.out_err + dglob, err);
        }
      }
    }
    prim::sync();
    prim::trace(t, 7);
  }

finish:
  // The last workgroup out resets the counters for the next launch and clears
  // a rotating window of descriptors so that no stale descriptor can ever
  // carry a matching epoch.
  prim::sync();
  if (tid == 0) {
    prim::fence();
    uint32_t old = prim::add_agent32(&ws->done, 1u);
    sh.is_last = (old == prim::grid() - 1) ? 1u : 0u;
  }
  prim::sync();
  if (sh.is_last) {
    uint64_t nwin = (a.cap_tiles + kScrub - 1) / kScrub;
    uint64_t w0 = (uint64_t)(epoch % (uint32_t)(nwin ? nwin : 1)) * kScrub;
    for (uint64_t j = w0 + tid; j < w0 + kScrub && j < a.cap_tiles; j += kThreads) st_desc(ws, (int64_t)j, 0ull);
    prim::sync();
    if (tid == 0) {
      prim::st_agent32(&ws->ticket, 0u);
      prim::st_agent32(&ws->done, 0u);
      prim::st_agent32(&ws->epoch, epoch + 1u);
    }
  }
}

}  // namespace jsidx
