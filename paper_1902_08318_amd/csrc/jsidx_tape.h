// jsidx_tape.h -- stage 2's tape (Sec. 3, Fig. 2) from a document's structural
// index and scope links: 64-bit words tagged with a character in bits 56..63,
// numbers parsed (two words: 'l' and an int64, or 'd' and a binary64), strings
// normalized into a string buffer (a 32-bit length, then UTF-8), literals
// checked.  Once the index is known no token depends on another (Sec. 3.2), so
// every entry is handled by its own thread:
//   1. tape_count: each entry's first byte and the buffer bytes of each string
//      (decoded, not written) go to the workspace; the words (0 for ':' and
//      ',', 2 for a number, else 1) and bytes are summed per chunk of 4096
//      entries;
//   2. tape_scan: one workgroup turns the chunk sums into bases and writes the
//      root words, the sizes, and clears the flags;
//   3. tape_offsets: each entry's tape index (a scan inside the chunk);
//   4. tape_write: the words of brackets (with the tape index of their
//      partner, from the scope links) and strings; strings, and numbers with
//      literals, are queued densely for
//   5. tape_strings: strings decoded into the buffer, and
//   6. tape_numbers: literals checked, numbers converted; a double whose
//      rounding the fast conversion cannot decide is queued again for
//   7. tape_exact: the exact big-integer conversion.
// Splitting by kind keeps the lanes of a wave on the same path.
// Consecutive threads take consecutive entries (coalesced); the scans inside
// a chunk run over the chunk staged in LDS.
// Written on the same primitives as the other kernels, so that the CPU
// emulation of the tests runs this source too.
#pragma once

#include "jsidx_device.h"
#include "jsidx_docscan.h"

#ifndef JSIDX_CONSTANT
#define JSIDX_CONSTANT __constant__
#endif
#include "jsidx_pow5.h"

namespace jsidx {

constexpr uint32_t kErrNumber = 0x100u;
constexpr uint32_t kErrString = 0x200u;
constexpr uint32_t kErrLiteral = 0x400u;
constexpr int kTapeThreads = 256;
constexpr int kTapePer = 16;
constexpr int kTapeChunk = kTapeThreads * kTapePer;
constexpr uint32_t kTapeUnlinked = 0xFFFFFFFFu;
constexpr int kExactGroups = 64;      // workgroups of tape_exact
constexpr int kQueueGroups = 8192;    // at most this many workgroups for the string and number queues
constexpr int kExactThreads = 64;     // one wave each
constexpr int kMaxDigits = 800;       // significant digits kept by the exact path
constexpr int kBigLimbs = 300;        // 9600 bits per big integer

struct TapeArgs {
  const uint8_t* buf;
  uint64_t len;
  const uint32_t* idx;
  uint32_t n;
  uint32_t nchunks;
  const uint32_t* match;
  uint64_t* tape;
  uint8_t* str;
  uint64_t* tape_n;
  uint64_t* str_n;
  uint32_t* err;
  // workspace
  uint64_t* chunk_sum;  // 2 per chunk: words, buffer bytes; then their bases
  uint32_t* sbytes;     // per entry: buffer bytes of a string, else 0
  uint8_t* kb;          // per entry: its first byte
  uint32_t* toff;       // per entry: tape index of its first word
  uint32_t* qcount;     // queue lengths: [0] exact conversions, [1] strings, [2] numbers
  uint32_t* queue;      // entries for the exact conversion
  uint64_t* squeue;     // strings: entry and buffer offset
  uint32_t* nqueue;     // numbers: entry
  // batches (jsidx_tape_batch): the documents' entries laid end to end as
  // "virtual" entries (an empty document gets one placeholder entry, so that
  // its two root words have an owner), every position absolute in buf, and
  // each document's tape and strings laid end to end in the outputs
  const uint64_t* offsets;  // ndocs + 1
  const uint32_t* dn;       // per document: its entry count (idx and match at + offsets[d])
  uint32_t ndocs;
  uint32_t cap;             // virtual entries the workspace holds
  uint64_t tape_cap, str_cap;  // words and bytes the outputs hold
  uint32_t* vn;             // [0] virtual entries, [1] their chunks, [2] 1 if the outputs hold the
                            // batch, [3] 1 if the batch is over the workspace's capacity
  uint64_t* part;           // per 2048 documents: entry sum, then base
  uint64_t* tot;            // total words and string bytes
  uint32_t* vstart;         // ndocs + 1: first virtual entry of each document
  uint32_t* docid;          // per virtual entry
  uint64_t* vpos;           // per virtual entry: absolute position of its first byte
  uint8_t* vflag;           // per virtual entry: kVFirst, kVLast, kVEmpty
  uint64_t* dbase;          // per document: first word of its tape, first byte of its strings
  uint64_t* out_pos;        // per document: tape start, tape words, string start, string bytes
};

constexpr uint32_t kVFirst = 1u, kVLast = 2u, kVEmpty = 4u;
constexpr uint32_t kTapeErrCapacity = 0x80000000u;

// Workspace layout of a batch (byte offsets; host side).
struct TapeBatchLayout {
  uint64_t vn, tot, qcount, part, vstart, docid, vpos, vflag, dbase, chunk_sum, sbytes, kb, toff, queue, squeue,
      nqueue, total;
};
inline TapeBatchLayout tape_batch_layout(uint64_t cap, uint64_t maxdocs) {
  const uint64_t nc = (cap + kTapeChunk - 1) / kTapeChunk;
  TapeBatchLayout L;
  uint64_t o = 0;
  auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  L.vn = o; o = al(o + 16);
  L.tot = o; o = al(o + 16);
  L.qcount = o; o = al(o + 16);
  L.part = o; o = al(o + (docscan_groups(maxdocs) + 1) * 8);
  L.vstart = o; o = al(o + (maxdocs + 1) * 4);
  L.docid = o; o = al(o + cap * 4);
  L.vpos = o; o = al(o + cap * 8);
  L.vflag = o; o = al(o + cap);
  L.dbase = o; o = al(o + maxdocs * 16);
  L.chunk_sum = o; o = al(o + nc * 16);
  L.sbytes = o; o = al(o + cap * 4);
  L.kb = o; o = al(o + cap);
  L.toff = o; o = al(o + cap * 4);
  L.queue = o; o = al(o + cap * 4);
  L.squeue = o; o = al(o + cap * 16);
  L.nqueue = o; o = al(o + cap * 4);
  L.total = o;
  return L;
}

struct TapeLayout {
  uint64_t chunk_sum, sbytes, kb, toff, qcount, queue, squeue, nqueue, total;
};
inline uint64_t tape_align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }
inline TapeLayout tape_layout(uint64_t n) {
  const uint64_t nc = (n + kTapeChunk - 1) / kTapeChunk;
  TapeLayout L;
  uint64_t o = 0;
  L.chunk_sum = o; o = tape_align256(o + nc * 16);
  L.sbytes = o; o = tape_align256(o + n * 4);
  L.kb = o; o = tape_align256(o + n);
  L.toff = o; o = tape_align256(o + n * 4);
  L.qcount = o; o = tape_align256(o + 16);
  L.queue = o; o = tape_align256(o + n * 4);
  L.squeue = o; o = tape_align256(o + n * 16);
  L.nqueue = o; o = tape_align256(o + n * 4);
  L.total = o;
  return L;
}

JSIDX_DEV uint32_t tape_tid() { return prim::wave_id() * 64u + prim::lane(); }

JSIDX_DEV uint32_t byte_at(const TapeArgs& a, uint64_t p) { return p < a.len ? prim::load1(a.buf + p) : 0u; }

// The first byte of entry i (0 if its position is not inside the document).
JSIDX_DEV uint32_t entry_byte(const TapeArgs& a, uint32_t i) {
  return byte_at(a, prim::load4(reinterpret_cast<const uint8_t*>(a.idx + i)));
}

JSIDX_DEV bool is_lit_start(uint32_t b) { return b == 't' || b == 'f' || b == 'n'; }

// The 32 bytes from the aligned word holding byte p on, loaded together into
// registers (eight word loads in flight), so that a short atom costs one
// memory round trip instead of one per byte.  Bytes past the window, or all
// bytes when it would leave the document, are loaded one by one; outside the
// document they read as 0.
struct Window {
  const uint8_t* buf;
  uint64_t len;
  uint64_t base;  // ~0: no window
  uint64_t q0, q1, q2, q3;
};
JSIDX_DEV Window window_at(const uint8_t* buf, uint64_t len, uint64_t p) {
  Window w{buf, len, ~0ull, 0, 0, 0, 0};
  const uint32_t off = (uint32_t)(reinterpret_cast<uintptr_t>(buf + p) & 3u);
  if (p < off || p - off + 32 > len) return w;
  w.base = p - off;
  uint32_t v[8];
#pragma unroll
  for (int j = 0; j < 8; j++) v[j] = prim::load4(buf + w.base + 4 * j);
  w.q0 = ((uint64_t)v[1] << 32) | v[0];
  w.q1 = ((uint64_t)v[3] << 32) | v[2];
  w.q2 = ((uint64_t)v[5] << 32) | v[4];
  w.q3 = ((uint64_t)v[7] << 32) | v[6];
  return w;
}
// One of four values by mask arithmetic (a chain of selects may be turned
// into an indexed array in private memory).
JSIDX_DEV uint64_t pick4(uint64_t a0, uint64_t a1, uint64_t a2, uint64_t a3, uint32_t i) {
  return (a0 & (0ull - (uint64_t)(i == 0))) | (a1 & (0ull - (uint64_t)(i == 1))) |
         (a2 & (0ull - (uint64_t)(i == 2))) | (a3 & (0ull - (uint64_t)(i == 3)));
}
JSIDX_DEV uint32_t win_byte(const Window& w, uint64_t p) {
  if (p >= w.len) return 0u;
  const uint64_t d = p - w.base;
  if (p < w.base || d >= 32) return prim::load1(w.buf + p);
  const uint64_t q = pick4(w.q0, w.q1, w.q2, w.q3, (uint32_t)(d >> 3));
  return (uint32_t)(q >> (8 * (d & 7u))) & 0xFFu;
}

// Tape words of an entry by its first byte.
JSIDX_DEV uint32_t words_of(uint32_t b) {
  if (b == ':' || b == ',') return 0;
  if (b == '{' || b == '}' || b == '[' || b == ']' || b == '"' || is_lit_start(b)) return 1;
  return 2;  // a number (or an invalid atom, which is a number error)
}

// An atom ends at white space, a structural character or the document's end.
JSIDX_DEV bool ends_atom(const Window& w, uint64_t p) {
  if (p >= w.len) return true;
  const uint32_t c = win_byte(w, p);
  return c == ' ' || c == '\t' || c == '\n' || c == '\r' || c == ',' || c == ':' || c == '[' || c == ']' ||
         c == '{' || c == '}';
}

// ---- Strings (Sec. 3.2.2) ---------------------------------------------------
JSIDX_DEV int32_t hex_digit(uint32_t c) {
  if (c >= '0' && c <= '9') return (int32_t)(c - '0');
  if (c >= 'a' && c <= 'f') return (int32_t)(c - 'a' + 10);
  if (c >= 'A' && c <= 'F') return (int32_t)(c - 'A' + 10);
  return -1;
}

// Four hex digits at p, or -1.
JSIDX_DEV int32_t hex_quad(const TapeArgs& a, uint64_t p) {
  if (p + 4 > a.len) return -1;
  int32_t v = 0;
  for (int k = 0; k < 4; k++) {
    const int32_t h = hex_digit(prim::load1(a.buf + p + k));
    if (h < 0) return -1;
    v = v * 16 + h;
  }
  return v;
}

template <bool WRITE>
JSIDX_DEV void emit(uint8_t* out, uint32_t* k, uint32_t v) {
  if constexpr (WRITE) prim::st_byte(out + *k, v);
  ++*k;
}

constexpr uint32_t kDeferred = 0x80000000u;  // string_run: the budget ran out

// The escape whose backslash is at *p: its bytes (\uXXXX and surrogate pairs
// as UTF-8) written if `writer`, *p and *k past it.  Returns 0 or kErrString.
template <bool WRITE>
JSIDX_DEV uint32_t escape_at(const TapeArgs& a, uint64_t* pp, uint8_t* out, uint32_t* kk, bool writer) {
  uint64_t p = *pp;
  uint32_t k = *kk;
  auto put = [&](uint32_t v) {
    if constexpr (WRITE) {
      if (writer) prim::st_byte(out + k, v);
    }
    k++;
  };
  if (p + 1 >= a.len) return kErrString;
  const uint32_t e = prim::load1(a.buf + p + 1);
  p += 2;
  uint32_t v = 0xFFFFFFFFu;
  switch (e) {
    case '"': v = '"'; break;
    case '\\': v = '\\'; break;
    case '/': v = '/'; break;
    case 'b': v = 0x08u; break;
    case 'f': v = 0x0Cu; break;
    case 'n': v = 0x0Au; break;
    case 'r': v = 0x0Du; break;
    case 't': v = 0x09u; break;
    default: break;
  }
  if (v != 0xFFFFFFFFu) {
    put(v);
  } else {
    if (e != 'u') return kErrString;
    const int32_t u = hex_quad(a, p);
    if (u < 0) return kErrString;
    p += 4;
    uint32_t cp = (uint32_t)u;
    if (cp >= 0xDC00u && cp <= 0xDFFFu) return kErrString;  // a low surrogate first
    if (cp >= 0xD800u && cp <= 0xDBFFu) {
      if (p + 2 > a.len || prim::load1(a.buf + p) != '\\' || prim::load1(a.buf + p + 1) != 'u') return kErrString;
      const int32_t lo = hex_quad(a, p + 2);
      if (lo < 0xDC00 || lo > 0xDFFF) return kErrString;
      p += 6;
      cp = 0x10000u + ((cp - 0xD800u) << 10) + ((uint32_t)lo - 0xDC00u);
    }
    if (cp < 0x80u) {
      put(cp);
    } else if (cp < 0x800u) {
      put(0xC0u | (cp >> 6));
      put(0x80u | (cp & 0x3Fu));
    } else if (cp < 0x10000u) {
      put(0xE0u | (cp >> 12));
      put(0x80u | ((cp >> 6) & 0x3Fu));
      put(0x80u | (cp & 0x3Fu));
    } else {
      put(0xF0u | (cp >> 18));
      put(0x80u | ((cp >> 12) & 0x3Fu));
      put(0x80u | ((cp >> 6) & 0x3Fu));
      put(0x80u | (cp & 0x3Fu));
    }
  }
  *pp = p;
  *kk = k;
  return 0;
}

// One thread's part of a string: from byte *p on (inside the string, *k bytes
// already out) up to the closing quote, with at most `budget` steps over
// whole plain blocks.  Returns 0 (closed), kErrString (a byte below 0x20, a
// bad escape, no closing quote; the count then stops there, the same in
// both modes) or kDeferred (*p and *k say where it stopped).
template <bool WRITE>
JSIDX_DEV uint32_t string_run(const TapeArgs& a, uint64_t* pp, uint8_t* out, uint32_t* kk, uint32_t budget) {
  uint64_t p = *pp;
  uint32_t k = *kk;
  uint32_t err = 0;
  uint32_t steps = 0;
  for (;;) {
    // 16 bytes from the aligned word holding p on (four loads in flight): the
    // plain bytes up to the first quote, backslash or control byte are taken
    // from registers; that byte is handled below
    const uint32_t off = (uint32_t)(reinterpret_cast<uintptr_t>(a.buf + p) & 3u);
    if (p >= off && p - off + 16 <= a.len) {
      const uint64_t pb = p - off;
      const uint32_t x0 = prim::load4(a.buf + pb), x1 = prim::load4(a.buf + pb + 4);
      const uint32_t x2 = prim::load4(a.buf + pb + 8), x3 = prim::load4(a.buf + pb + 12);
      // the lowest flagged byte of a word is exact (a borrow only runs upward)
      auto hits = [](uint32_t v) {
        const uint32_t q2 = v ^ 0x22222222u, b2 = v ^ 0x5C5C5C5Cu;
        return (((q2 - 0x01010101u) & ~q2) | ((b2 - 0x01010101u) & ~b2) | ((v - 0x20202020u) & ~v)) & 0x80808080u;
      };
      const uint32_t h0 = hits(x0) & (0xFFFFFFFFu << (8 * off)), h1 = hits(x1), h2 = hits(x2), h3 = hits(x3);
      // the first special byte at or after p, in the block (16: none)
      const uint32_t first = h0 ? (uint32_t)__builtin_ctz(h0) / 8
                           : h1 ? 4 + (uint32_t)__builtin_ctz(h1) / 8
                           : h2 ? 8 + (uint32_t)__builtin_ctz(h2) / 8
                           : h3 ? 12 + (uint32_t)__builtin_ctz(h3) / 8 : 16u;
      // bytes [off, first) are plain: whole words where the destination is
      // aligned (taken from the window shifted as a 128-bit value), single
      // bytes around them
      if constexpr (WRITE) {
        const uint64_t lo64 = ((uint64_t)x1 << 32) | x0, hi64 = ((uint64_t)x3 << 32) | x2;
        const uint32_t cnt = first - off;
        const uint32_t da = (uint32_t)(reinterpret_cast<uintptr_t>(out + k) & 3u);
        uint32_t m0 = (4u - da) & 3u;
        if (m0 > cnt) m0 = cnt;
        const uint32_t nw = (cnt - m0) / 4;
        for (uint32_t m = 0; m < cnt; m++) {
          if (m == m0 && nw) m += 4 * nw;  // the words below
          if (m >= cnt) break;
          const uint32_t idx = off + m;
          prim::st_byte(out + k + m, (uint32_t)((idx < 8 ? lo64 >> (8 * idx) : hi64 >> (8 * (idx - 8))) & 0xFFu));
        }
        if (nw) {
          const uint32_t r = 8 * (off + m0);  // below 64: off and m0 are at most 3
          const uint64_t slo = r ? (lo64 >> r) | (hi64 << (64 - r)) : lo64, shi = hi64 >> r;
          uint32_t* dw = reinterpret_cast<uint32_t*>(out + k + m0);
          prim::st_out(dw, (uint32_t)slo);
          if (nw > 1) prim::st_out(dw + 1, (uint32_t)(slo >> 32));
          if (nw > 2) prim::st_out(dw + 2, (uint32_t)shi);
          if (nw > 3) prim::st_out(dw + 3, (uint32_t)(shi >> 32));
        }
      }
      k += first - off;
      p = pb + first;
      if (first == 16) {
        if (++steps >= budget) { err = kDeferred; break; }
        continue;
      }
      // the special byte is in the registers: a closing quote ends the string
      // without another load
      const uint32_t fw = first < 8 ? (first < 4 ? x0 : x1) : (first < 12 ? x2 : x3);
      if (((fw >> (8 * (first & 3u))) & 0xFFu) == '"') break;
    }
    if (p >= a.len) { err = kErrString; break; }
    const uint32_t c = prim::load1(a.buf + p);
    if (c == '"') break;
    if (c < 0x20u) { err = kErrString; break; }
    if (c != '\\') {
      emit<WRITE>(out, &k, c);
      p++;
      continue;
    }
    err = escape_at<WRITE>(a, &p, out, &k, true);
    if (err) break;
  }
  *pp = p;
  *kk = k;
  return err;
}

// The rest of a string by the whole wave (every lane calls it with the same
// arguments): 64 bytes per step, one per lane, the first quote, backslash or
// control byte found by ballot; the plain bytes before it are written by
// their lanes (coalesced), an escape is decoded by every lane and written by
// lane 0.  Returns 0 or kErrString; *k as string_run.
template <bool WRITE>
JSIDX_DEV uint32_t string_wave(const TapeArgs& a, uint64_t p, uint8_t* out, uint32_t* kk) {
  const uint32_t lane = prim::lane();
  uint32_t k = *kk;
  uint32_t err = 0;
  for (;;) {
    const uint64_t pos = p + lane;
    const uint32_t c = pos < a.len ? prim::load1(a.buf + pos) : 0x100u;
    const bool special = c >= 0x100u || c == '"' || c == '\\' || c < 0x20u;
    const uint64_t m = prim::ballot(special);
    const uint32_t f = m ? (uint32_t)__builtin_ctzll(m) : 64u;
    if constexpr (WRITE) {
      if (lane < f) prim::st_byte(out + k + lane, c);
    }
    k += f;
    p += f;
    if (f == 64) continue;
    const uint32_t c0 = prim::readlane(c, (int)f);  // the special byte, the same for every lane
    if (c0 == '"') break;
    if (c0 >= 0x100u || c0 < 0x20u) { err = kErrString; break; }
    err = escape_at<WRITE>(a, &p, out, &k, lane == 0);
    if (err) break;
  }
  *kk = k;
  return err;
}

// Strings of a wave, each lane's string opening at q (if `has`): its bytes
// after normalization (escapes decoded, \uXXXX and surrogate pairs as UTF-8)
// to out (WRITE) and their count to *n.  A byte below 0x20, an unknown
// escape, a malformed or lone surrogate, or no closing quote is an error (the
// count then stops there, the same in both modes).  Each lane runs its own
// string for kStringSteps blocks; the strings that outrun it are then
// finished one after another by the whole wave.  Every lane of the wave must
// call this.
constexpr uint32_t kStringSteps = 2;
template <bool WRITE>
JSIDX_DEV uint32_t wave_strings(const TapeArgs& a, bool has, uint64_t q, uint8_t* out, uint32_t* n) {
  uint64_t p = q + 1;
  uint32_t k = 0;
  uint32_t err = has ? string_run<WRITE>(a, &p, out, &k, kStringSteps) : 0u;
  uint64_t m = prim::ballot(err == kDeferred);
  while (m) {
    const int L = __builtin_ctzll(m);
    m &= m - 1;
    const uint64_t pL = ((uint64_t)prim::readlane((uint32_t)(p >> 32), L) << 32) | prim::readlane((uint32_t)p, L);
    uint32_t kL = prim::readlane(k, L);
    uint8_t* outL = nullptr;
    if constexpr (WRITE) {
      const uint64_t o = reinterpret_cast<uintptr_t>(out);
      outL = reinterpret_cast<uint8_t*>(((uint64_t)prim::readlane((uint32_t)(o >> 32), L) << 32) |
                                        prim::readlane((uint32_t)o, L));
    }
    // the lane's own document bound (a batch's lanes may hold different documents)
    TapeArgs aL = a;
    aL.len = ((uint64_t)prim::readlane((uint32_t)(a.len >> 32), L) << 32) | prim::readlane((uint32_t)a.len, L);
    const uint32_t e = string_wave<WRITE>(aL, pL, outL, &kL);
    if ((int)prim::lane() == L) {
      k = kL;
      err = e;
    }
  }
  *n = k;
  return err;
}

// ---- Literals ---------------------------------------------------------------
JSIDX_DEV bool literal_ok(const TapeArgs& a, uint64_t p, uint32_t first) {
  // true, false, null by their bytes (little-endian words)
  const uint32_t L = first == 'f' ? 5u : 4u;
  if (p + L > a.len) return false;
  const Window w = window_at(a.buf, a.len, p);
  uint64_t v = 0;
  for (uint32_t k = 0; k < L; k++) v |= (uint64_t)win_byte(w, p + k) << (8 * k);
  const uint64_t want = first == 't' ? 0x65757274ull : first == 'n' ? 0x6C6C756Eull : 0x65736C6166ull;
  return v == want && ends_atom(w, p + L);
}

// ---- Numbers (Sec. 3.2.1) ---------------------------------------------------
// The number grammar: an optional minus, 0 or a nonzero digit and digits, an
// optional fraction ('.' and digits), an optional exponent (e or E, a sign,
// digits); it must end the atom.  The decimal value is w * 10^q, with w the
// first 19 significant digits; trunc says a nonzero digit was dropped (the
// value then lies strictly between w * 10^q and (w + 1) * 10^q).
struct NumText {
  bool ok, neg, is_int, trunc;
  uint32_t int_digits;  // digits of the integer part
  uint64_t w;
  int64_t q;
};

JSIDX_DEV bool is_digit(uint32_t c) { return c - '0' <= 9u; }

JSIDX_DEV NumText scan_number(const TapeArgs& a, uint64_t p) {
  NumText t{false, false, true, false, 0, 0, 0};
  const Window w = window_at(a.buf, a.len, p);
  uint32_t nd = 0;  // significant digits in w
  int64_t q = 0;
  uint32_t c = win_byte(w, p);
  if (c == '-') {
    t.neg = true;
    c = win_byte(w, ++p);
  }
  if (!is_digit(c)) return t;
  if (c == '0') {
    t.int_digits = 1;
    c = win_byte(w, ++p);
  } else {
    while (p < a.len && is_digit(c)) {
      t.int_digits++;
      if (nd < 19) {
        t.w = t.w * 10 + (c - '0');
        nd++;
      } else {
        q++;  // a dropped digit of the integer part scales the rest
        t.trunc = t.trunc || c != '0';
      }
      c = win_byte(w, ++p);
    }
  }
  if (p < a.len && c == '.') {
    t.is_int = false;
    c = win_byte(w, ++p);
    if (!(p < a.len && is_digit(c))) return t;
    while (p < a.len && is_digit(c)) {
      if (nd == 0 && c == '0') {
        q--;  // a leading zero of the fraction
      } else if (nd < 19) {
        t.w = t.w * 10 + (c - '0');
        nd++;
        q--;
      } else {
        t.trunc = t.trunc || c != '0';
      }
      c = win_byte(w, ++p);
    }
  }
  if (p < a.len && (c == 'e' || c == 'E')) {
    t.is_int = false;
    c = win_byte(w, ++p);
    bool eneg = false;
    if (p < a.len && (c == '+' || c == '-')) {
      eneg = c == '-';
      c = win_byte(w, ++p);
    }
    if (!(p < a.len && is_digit(c))) return t;
    int64_t e = 0;
    while (p < a.len && is_digit(c)) {
      if (e < 100000000) e = e * 10 + (c - '0');
      c = win_byte(w, ++p);
    }
    q += eneg ? -e : e;
  }
  t.q = q;
  t.ok = ends_atom(w, p);
  return t;
}

// 64 x 64 -> 128-bit product.
JSIDX_DEV void mul_64(uint64_t x, uint64_t y, uint64_t* hi, uint64_t* lo) {
  const uint64_t x0 = (uint32_t)x, x1 = x >> 32, y0 = (uint32_t)y, y1 = y >> 32;
  const uint64_t p00 = x0 * y0, p01 = x0 * y1, p10 = x1 * y0, p11 = x1 * y1;
  const uint64_t mid = (p00 >> 32) + (uint32_t)p01 + (uint32_t)p10;
  *lo = (mid << 32) | (uint32_t)p00;
  *hi = p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
}

constexpr uint64_t kInfBits = 0x7FF0000000000000ull;
enum : int { kConvOk = 0, kConvInf = 1, kConvUndecided = 2 };

// The binary64 nearest to w * 10^q (w > 0), ties to even, when a 128-bit
// approximation decides it.  w is normalized to 64 bits and multiplied by
// the table's 128-bit T with 5^q ~ T * 2^k; of the 192-bit product the top
// 128 bits P are kept, and w * 10^q = P * 2^(64 + k + q - lz) up to an error
// below 2 units of P's last bit (the dropped low word, and T's own rounding,
// downward for q >= 0 and upward for q < 0).  The rounding position is the
// 53rd bit below P's top bit, or the bit of 2^-1074 for subnormal results.
// The result is undecided when the bits below that position are within 3
// units of exactly half.
JSIDX_DEV int fast_double(uint64_t w, int64_t q, uint64_t* bits) {
  if (q > kPow5Max) return kConvInf;       // at least 10^309
  if (q < kPow5Min) { *bits = 0; return kConvOk; }  // below 10^-323 / 2
  const Pow5 T = kPow5[q - kPow5Min];
  const int lz = __builtin_clzll(w);
  const uint64_t wn = w << lz;
  uint64_t a1, a0, b1, b0;
  mul_64(wn, T.lo, &a1, &a0);
  mul_64(wn, T.hi, &b1, &b0);
  const uint64_t plo = b0 + a1;
  const uint64_t phi = b1 + (plo < b0 ? 1u : 0u);
  const int msb = (phi >> 63) ? 127 : 126;
  const int64_t base = 64 + (int64_t)T.k + q - lz;  // value = P * 2^base
  const int64_t e2 = msb + base;                     // exponent of the top bit
  if (e2 >= 1024) return kConvInf;
  const int64_t rp = e2 >= -1022 ? msb - 52 : -1074 - base;  // bit of the result's last place
  if (rp >= 130) { *bits = 0; return kConvOk; }  // below a quarter of 2^-1074
  if (rp >= 128) return kConvUndecided;
  // rp in [74, 127]: the result bits are in phi; R = P mod 2^rp
  const int sh = (int)rp - 64;
  uint64_t m = phi >> sh;
  const uint64_t rhi = phi & ((1ull << sh) - 1u), rlo = plo;
  const uint64_t hhi = 1ull << (sh - 1);  // half = 2^(rp - 1), low word 0
  if ((rhi == hhi && rlo <= 3u) || (rhi + 1u == hhi && rlo >= ~0ull - 2u)) return kConvUndecided;
  const bool up = rhi > hhi || (rhi == hhi && rlo != 0u);
  m += up ? 1u : 0u;
  uint64_t b;
  if (e2 >= -1022) b = ((uint64_t)(e2 + 1023) << 52) + (m - (1ull << 52));  // m in [2^52, 2^53]
  else b = m;                                                               // subnormal, m <= 2^52
  if (b >= kInfBits) return kConvInf;
  *bits = b;
  return kConvOk;
}

// ---- The exact conversion (rare: undecided by fast_double) -----------------
struct Big {
  uint32_t d[kBigLimbs];  // little-endian limbs
  int n;                  // limbs in use (no leading zero limb)
};

JSIDX_DEV void big_set(Big& x, uint32_t v) {
  x.n = v ? 1 : 0;
  x.d[0] = v;
}
JSIDX_DEV void big_mul_add(Big& x, uint32_t m, uint32_t add) {
  uint64_t carry = add;
  for (int i = 0; i < x.n; i++) {
    const uint64_t t = (uint64_t)x.d[i] * m + carry;
    x.d[i] = (uint32_t)t;
    carry = t >> 32;
  }
  if (carry && x.n < kBigLimbs) x.d[x.n++] = (uint32_t)carry;
}
JSIDX_DEV void big_mul_pow5(Big& x, int64_t e) {
  while (e >= 13) {
    big_mul_add(x, 1220703125u, 0);  // 5^13
    e -= 13;
  }
  uint32_t m = 1;
  while (e-- > 0) m *= 5;
  if (m != 1) big_mul_add(x, m, 0);
}
JSIDX_DEV int64_t big_bits(const Big& x) {
  return x.n ? 32 * (int64_t)(x.n - 1) + (32 - __builtin_clz(x.d[x.n - 1])) : 0;
}
JSIDX_DEV void big_shl(Big& x, int64_t s) {
  if (!x.n || s <= 0) return;
  const int w = (int)(s / 32), b = (int)(s % 32);
  int nn = x.n + w + 1;
  if (nn > kBigLimbs) nn = kBigLimbs;
  for (int i = nn - 1; i >= 0; i--) {
    const int j = i - w;
    const uint32_t hi = (j >= 0 && j < x.n) ? x.d[j] : 0u;
    const uint32_t lo = (j - 1 >= 0 && j - 1 < x.n) ? x.d[j - 1] : 0u;
    x.d[i] = b ? (hi << b) | (lo >> (32 - b)) : hi;
  }
  x.n = nn;
  while (x.n && !x.d[x.n - 1]) x.n--;
}
JSIDX_DEV int big_cmp(const Big& x, const Big& y) {
  if (x.n != y.n) return x.n < y.n ? -1 : 1;
  for (int i = x.n - 1; i >= 0; i--)
    if (x.d[i] != y.d[i]) return x.d[i] < y.d[i] ? -1 : 1;
  return 0;
}
JSIDX_DEV void big_sub(Big& x, const Big& y) {  // x -= y, x >= y
  int64_t borrow = 0;
  for (int i = 0; i < x.n; i++) {
    const int64_t t = (int64_t)x.d[i] - (i < y.n ? (int64_t)y.d[i] : 0) - borrow;
    x.d[i] = (uint32_t)t;
    borrow = t < 0 ? 1 : 0;
  }
  while (x.n && !x.d[x.n - 1]) x.n--;
}
// The top 64 bits of x (x != 0; its top bit becomes bit 63) and whether any
// bit below them is set.
JSIDX_DEV uint64_t big_top64(const Big& x, bool* sticky) {
  const int64_t L = big_bits(x);
  uint64_t r = 0;
  bool s = false;
  for (int64_t b = L - 1; b >= 0; b--) {
    const uint32_t bit = (x.d[b / 32] >> (b % 32)) & 1u;
    if (L - 1 - b < 64) r |= (uint64_t)bit << (63 - (L - 1 - b));
    else if (bit) { s = true; break; }
  }
  *sticky = s;
  return r;
}

// Round m * 2^(e2 - 63) (m with its top bit set), plus a nonzero tail if
// sticky, to binary64; kConvInf if it overflows.
JSIDX_DEV int round_to_double(uint64_t m, int64_t e2, bool sticky, uint64_t* bits) {
  if (e2 > 1023) return kConvInf;
  const int64_t sh = e2 >= -1022 ? 11 : 11 + (-1022 - e2);  // bits of m below the last place
  uint64_t r;
  bool rb, rest;
  if (sh >= 66) {
    *bits = 0;
    return kConvOk;
  }
  if (sh >= 64) {
    r = 0;
    rb = sh == 64 && (m >> 63);
    rest = (sh == 64 ? (m << 1) != 0 : m != 0) || sticky;
  } else {
    r = m >> sh;
    rb = (m >> (sh - 1)) & 1u;
    rest = (m & ((1ull << (sh - 1)) - 1u)) != 0 || sticky;
  }
  if (rb && (rest || (r & 1u))) r++;
  const uint64_t b = e2 >= -1022 ? ((uint64_t)(e2 + 1023) << 52) + (r - (1ull << 52)) : r;
  if (b >= kInfBits) return kConvInf;
  *bits = b;
  return kConvOk;
}

// The exact binary64 of the number text at p (grammar already checked): all
// significant digits D (the first kMaxDigits, then a final 1 standing for any
// nonzero rest) with x = D * 10^e.  For e >= 0, D * 5^e is exact and x its
// multiple by 2^e; for e < 0 the quotient of D * 2^t by 5^-e is taken by
// binary long division to 66 bits, x = quotient * 2^(-t + e), and the
// remainder is the sticky tail.
JSIDX_DEV int exact_double(const TapeArgs& a, uint64_t p, Big& D, Big& V, Big& S, uint64_t* bits) {
  big_set(D, 0);
  int64_t e = 0;
  int nd = 0;
  bool drop = false;
  uint32_t chunk = 0, chunk_mul = 1;
  auto digit = [&](uint32_t dv) {
    chunk = chunk * 10 + dv;
    chunk_mul *= 10;
    nd++;
    if (chunk_mul == 1000000000u) {
      big_mul_add(D, chunk_mul, chunk);
      chunk = 0;
      chunk_mul = 1;
    }
  };
  uint32_t c = byte_at(a, p);
  if (c == '-') c = byte_at(a, ++p);
  while (p < a.len && is_digit(c)) {
    if (nd == 0 && c == '0') {
      // the single leading zero of the integer part
    } else if (nd < kMaxDigits) {
      digit(c - '0');
    } else {
      e++;
      drop = drop || c != '0';
    }
    c = byte_at(a, ++p);
  }
  if (p < a.len && c == '.') {
    c = byte_at(a, ++p);
    while (p < a.len && is_digit(c)) {
      if (nd == 0 && c == '0') {
        e--;
      } else if (nd < kMaxDigits) {
        digit(c - '0');
        e--;
      } else {
        drop = drop || c != '0';
      }
      c = byte_at(a, ++p);
    }
  }
  if (chunk_mul > 1) big_mul_add(D, chunk_mul, chunk);
  if (drop) {  // strictly between D * 10^e and (D + 1) * 10^e
    big_mul_add(D, 10, 1);
    e--;
  }
  if (p < a.len && (c == 'e' || c == 'E')) {
    c = byte_at(a, ++p);
    bool eneg = false;
    if (c == '+' || c == '-') {
      eneg = c == '-';
      c = byte_at(a, ++p);
    }
    int64_t x = 0;
    while (p < a.len && is_digit(c)) {
      if (x < 100000000) x = x * 10 + (c - '0');
      c = byte_at(a, ++p);
    }
    e += eneg ? -x : x;
  }
  if (D.n == 0) { *bits = 0; return kConvOk; }
  const int64_t dbits = big_bits(D);
  if (e >= 0) {
    if (dbits + 3 * e > 2000) return kConvInf;  // 10^e > 2^(3e): far beyond the range
    big_mul_pow5(D, e);
    bool sticky;
    const uint64_t m = big_top64(D, &sticky);
    return round_to_double(m, big_bits(D) - 1 + e, sticky, bits);
  }
  const int64_t c5 = -e;
  if (dbits - 2 * c5 < -1200) { *bits = 0; return kConvOk; }  // 10^e < 2^(-3.3 c5): far below 2^-1075
  big_set(V, 1);
  big_mul_pow5(V, c5);
  // shift so that the quotient has 66 bits: bits(N) - bits(V') == 65
  const int64_t t = big_bits(V) - dbits + 65;
  if (t >= 0) big_shl(D, t);
  else big_shl(V, -t);
  uint64_t qhi = 0, qlo = 0;  // the quotient, below 2^66
  for (int j = 66; j >= 0; j--) {
    for (int i = 0; i < V.n; i++) S.d[i] = V.d[i];
    S.n = V.n;
    big_shl(S, j);
    if (big_cmp(D, S) >= 0) {
      big_sub(D, S);
      if (j >= 64) qhi |= 1ull << (j - 64);
      else qlo |= 1ull << j;
    }
  }
  const bool rem = D.n != 0;
  // normalize the quotient to 64 bits
  const int qb = qhi ? 64 + (64 - __builtin_clzll(qhi)) : 64 - __builtin_clzll(qlo);
  const int drop_bits = qb - 64;  // 0..3 (the quotient has at least 64 bits)
  const uint64_t m = drop_bits > 0 ? (qhi << (64 - drop_bits)) | (qlo >> drop_bits) : qlo;
  const bool sticky = rem || (drop_bits > 0 && (qlo & ((1ull << drop_bits) - 1u)) != 0);
  return round_to_double(m, (int64_t)qb - 1 - t + e, sticky, bits);
}

// ---- Kernels ------------------------------------------------------------------

struct TapeScanLds {
  uint64_t w[kTapeThreads];
  uint64_t s[kTapeThreads];
};
// A chunk staged in LDS: first bytes, buffer bytes (then their prefix in the
// chunk), tape indices.
template <bool BATCH>
struct TapeChunkT {
  TapeScanLds sc;
  uint32_t qbase[2];  // the workgroup's first slots in the string and number queues
  uint32_t S[kTapeChunk];
  uint32_t T[kTapeChunk];
  uint8_t K[kTapeChunk];
  uint8_t F[BATCH ? kTapeChunk : 4];  // batch flags of the entries
};

// Exclusive scan over the workgroup of two sums (ex: the threads before this
// one; all: every thread).
template <typename G>
JSIDX_DEV void group_scan2(G& g, uint32_t tid, uint64_t w, uint64_t s, uint64_t* wex, uint64_t* sex,
                           uint64_t* wall, uint64_t* sall) {
  g.w[tid] = w;
  g.s[tid] = s;
  prim::sync();
  for (uint32_t d = 1; d < (uint32_t)kTapeThreads; d <<= 1) {
    const uint64_t tw = tid >= d ? g.w[tid - d] : 0, ts = tid >= d ? g.s[tid - d] : 0;
    prim::sync();
    g.w[tid] += tw;
    g.s[tid] += ts;
    prim::sync();
  }
  *wex = g.w[tid] - w;
  *sex = g.s[tid] - s;
  *wall = g.w[kTapeThreads - 1];
  *sall = g.s[kTapeThreads - 1];
  prim::sync();
}

JSIDX_DEV uint64_t ld64(const uint64_t* p) {
  const uint2 v = prim::ld_pair(reinterpret_cast<const uint2*>(p));
  return ((uint64_t)v.y << 32) | v.x;
}
JSIDX_DEV void st64(uint64_t* p, uint64_t v) {
  prim::st_pair(reinterpret_cast<uint2*>(p), (uint32_t)v, (uint32_t)(v >> 32));
}

// Entry i's position (absolute for a batch) and the arguments to parse it
// with (for a batch, the bound is its document's end).
template <bool BATCH>
JSIDX_DEV uint64_t entry_pos(const TapeArgs& a, uint64_t i) {
  return BATCH ? ld64(a.vpos + i) : prim::load4(reinterpret_cast<const uint8_t*>(a.idx + i));
}
template <bool BATCH>
JSIDX_DEV uint32_t entry_doc(const TapeArgs& a, uint64_t i) {
  return BATCH ? prim::load4(reinterpret_cast<const uint8_t*>(a.docid + i)) : 0u;
}
template <bool BATCH>
JSIDX_DEV TapeArgs entry_args(const TapeArgs& a, uint32_t d) {
  TapeArgs r = a;
  if (BATCH) r.len = prim::load8(a.offsets + d + 1);
  return r;
}
template <bool BATCH>
JSIDX_DEV uint32_t n_of(const TapeArgs& a) { return BATCH ? prim::ld_agent32(a.vn) : a.n; }
template <bool BATCH>
JSIDX_DEV uint32_t nchunks_of(const TapeArgs& a) { return BATCH ? prim::ld_agent32(a.vn + 1) : a.nchunks; }
// Tape words of an entry with first byte b and batch flags f: its own, plus
// its document's root words if it is the document's first or last entry.
JSIDX_DEV uint32_t entry_words(uint32_t b, uint32_t f) {
  return words_of(b) + (f & kVFirst ? 1u : 0u) + (f & kVLast ? 1u : 0u);
}

// 1. First bytes and string sizes (thread t takes entries c * 4096 + t +
//    256 k), their sums per chunk.
template <bool BATCH>
JSIDX_DEVFN void tape_count(const TapeArgs& a) {
  TapeScanLds& g = prim::lds_object<TapeScanLds>();
  const uint32_t tid = tape_tid();
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  uint64_t w = 0, s = 0;
  for (int k = 0; k < kTapePer; k++) {  // every lane runs every step (wave_strings)
    const uint64_t i = (uint64_t)c * kTapeChunk + (uint64_t)k * kTapeThreads + tid;
    const bool in = i < n;
    const uint32_t f = BATCH && in ? prim::load1(a.vflag + i) : 0u;
    const TapeArgs la = entry_args<BATCH>(a, in ? entry_doc<BATCH>(a, i) : 0u);
    const uint64_t pos = in ? entry_pos<BATCH>(a, i) : 0u;
    const uint32_t b = !in ? 0u : (f & kVEmpty) ? (uint32_t)':' : byte_at(la, pos);
    uint32_t len = 0;
    (void)wave_strings<false>(la, in && b == '"', pos, nullptr, &len);
    if (!in) continue;
    const uint32_t sb = b == '"' ? 4 + len : 0u;
    prim::st_out(a.sbytes + i, sb);
    prim::st_byte(a.kb + i, b);
    w += entry_words(b, f);
    s += sb;
  }
  uint64_t wex, sex, wall, sall;
  group_scan2(g, tid, w, s, &wex, &sex, &wall, &sall);
  if (tid == 0) {
    st64(a.chunk_sum + 2 * (uint64_t)c, wall);
    st64(a.chunk_sum + 2 * (uint64_t)c + 1, sall);
  }
  prim::sync();
  }
}

// 2. Chunk bases (one workgroup), the root words, the sizes; flags cleared.
//    For a batch: the totals, checked against the outputs (a batch that does
//    not fit is not written: every document gets JSIDX_ERR_CAPACITY).
template <bool BATCH>
JSIDX_DEVFN void tape_scan(const TapeArgs& a) {
  TapeScanLds& g = prim::lds_object<TapeScanLds>();
  const uint32_t tid = tape_tid();
  const uint32_t nchunks = nchunks_of<BATCH>(a);
  const uint32_t per = (nchunks + kTapeThreads - 1) / kTapeThreads;
  const uint64_t lo = (uint64_t)tid * per;
  const uint64_t hi = lo + per < nchunks ? lo + per : nchunks;
  uint64_t w = 0, s = 0;
  for (uint64_t c = lo; c < hi; c++) {
    w += ld64(a.chunk_sum + 2 * c);
    s += ld64(a.chunk_sum + 2 * c + 1);
  }
  uint64_t wex, sex, wall, sall;
  group_scan2(g, tid, w, s, &wex, &sex, &wall, &sall);
  for (uint64_t c = lo; c < hi; c++) {
    const uint64_t cw = ld64(a.chunk_sum + 2 * c), cs = ld64(a.chunk_sum + 2 * c + 1);
    st64(a.chunk_sum + 2 * c, wex);
    st64(a.chunk_sum + 2 * c + 1, sex);
    wex += cw;
    sex += cs;
  }
  if (BATCH) {
    if (nchunks == 0) return;  // tape_batch_bases flagged the batch
    const bool fits = wall <= a.tape_cap && sall <= a.str_cap;
    if (!fits)
      for (uint32_t d = tid; d < a.ndocs; d += (uint32_t)kTapeThreads) prim::st_out(a.err + d, kTapeErrCapacity);
    if (tid == 0) {
      st64(a.tot, wall);
      st64(a.tot + 1, sall);
      prim::st_out(a.vn + 2, fits ? 1u : 0u);
    }
    return;
  }
  if (tid == 0) {
    const uint64_t last = wall + 1;  // the root words enclose the words of the entries
    st64(a.tape, ((uint64_t)'r' << 56) | last);
    st64(a.tape + last, (uint64_t)'r' << 56);
    st64(a.tape_n, last + 1);
    st64(a.str_n, sall);
    prim::st_out(a.err, 0u);
    for (int q = 0; q < 3; q++) prim::st_out(a.qcount + q, 0u);
  }
}

// Whether a batch's outputs hold it (kernels after tape_scan).
template <bool BATCH>
JSIDX_DEV bool batch_go(const TapeArgs& a) { return !BATCH || prim::ld_agent32(a.vn + 2) != 0u; }

// Stages chunk c (first bytes and string sizes, loaded coalesced) and turns
// them into each entry's tape index (T) and buffer offset (S) by a scan over
// the threads' runs of 16 entries.  (For a batch, T is the index of the
// entry's own first word, after its document's opening root word if it is
// the document's first entry; F holds the batch flags.)
template <bool BATCH>
JSIDX_DEV void stage_offsets(const TapeArgs& a, uint32_t n, TapeChunkT<BATCH>& g, uint32_t tid, uint32_t c) {
  const uint64_t c0 = (uint64_t)c * kTapeChunk;
  for (uint32_t j = tid; j < (uint32_t)kTapeChunk; j += kTapeThreads) {
    const bool in = c0 + j < n;
    g.K[j] = (uint8_t)(in ? prim::load1(a.kb + c0 + j) : ':');
    g.S[j] = in ? prim::load4(reinterpret_cast<const uint8_t*>(a.sbytes + c0 + j)) : 0u;
    if (BATCH) g.F[j] = (uint8_t)(in ? prim::load1(a.vflag + c0 + j) : 0u);
  }
  prim::sync();
  uint64_t w = 0, s = 0;
  for (int k = 0; k < kTapePer; k++) {
    const uint32_t j = tid * kTapePer + (uint32_t)k;
    w += BATCH ? entry_words(g.K[j], g.F[j]) : words_of(g.K[j]);
    s += g.S[j];
  }
  uint64_t wex, sex, wall, sall;
  group_scan2(g.sc, tid, w, s, &wex, &sex, &wall, &sall);
  uint64_t tw = (BATCH ? 0 : 1) + ld64(a.chunk_sum + 2 * (uint64_t)c) + wex;
  uint64_t ts = ld64(a.chunk_sum + 2 * (uint64_t)c + 1) + sex;
  for (int k = 0; k < kTapePer; k++) {
    const uint32_t j = tid * kTapePer + (uint32_t)k;
    const uint32_t sb = g.S[j];
    const uint32_t first = BATCH && (g.F[j] & kVFirst) ? 1u : 0u;
    if (BATCH && first && c0 + j < n) {
      // the document's bases: its opening root word and its first string byte
      const uint32_t d = prim::load4(reinterpret_cast<const uint8_t*>(a.docid + c0 + j));
      st64(a.dbase + 2 * (uint64_t)d, tw);
      st64(a.dbase + 2 * (uint64_t)d + 1, ts);
    }
    g.T[j] = (uint32_t)(tw + first);
    g.S[j] = (uint32_t)ts;  // the buffer offset's low word (see tape_write)
    tw += BATCH ? entry_words(g.K[j], g.F[j]) : words_of(g.K[j]);
    ts += sb;
  }
  prim::sync();
}

// 3. Each entry's tape index, stored coalesced.
template <bool BATCH>
JSIDX_DEVFN void tape_offsets(const TapeArgs& a) {
  TapeChunkT<BATCH>& g = prim::lds_object<TapeChunkT<BATCH>>();
  const uint32_t tid = tape_tid();
  if (!batch_go<BATCH>(a)) return;
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
    stage_offsets<BATCH>(a, n, g, tid, c);
    const uint64_t c0 = (uint64_t)c * kTapeChunk;
    for (uint32_t j = tid; j < (uint32_t)kTapeChunk; j += kTapeThreads) {
      if (c0 + j >= n) break;
      prim::st_out(a.toff + c0 + j, g.T[j]);
    }
    prim::sync();
  }
}

// Flags of a wave: one atomic per flag that some lane set (for a batch, one
// per lane with a flag, to its document's word).
template <bool BATCH>
JSIDX_DEV void or_flags(const TapeArgs& a, uint32_t err, uint32_t d) {
  const uint32_t lane = prim::lane();
  if (BATCH) {
    if (err) prim::or_agent32(a.err + d, err);
    return;
  }
  for (uint32_t f = kErrNumber; f <= kErrLiteral; f <<= 1)
    if (prim::ballot((err & f) != 0u) != 0ull && lane == 0) prim::or_agent32(a.err, f);
}

// Appends the lanes with `take` to queue q (one atomic per wave); returns
// this lane's slot.
JSIDX_DEV uint32_t wave_append(const TapeArgs& a, int q, bool take) {
  const uint64_t m = prim::ballot(take);
  uint32_t base = 0;
  if (prim::lane() == 0 && m) base = prim::add_agent32(a.qcount + q, (uint32_t)__builtin_popcountll(m));
  base = prim::readlane(base, 0);
  return base + prim::mbcnt(m);
}

// 3b. Each document's root words and its place in the outputs (batches; one
//     thread per document).
JSIDX_DEVFN void tape_batch_docs(const TapeArgs& a) {
  if (!batch_go<true>(a)) return;
  const uint32_t stride = prim::grid() * (uint32_t)kTapeThreads;
  const uint64_t tw = ld64(a.tot), ts = ld64(a.tot + 1);
  for (uint32_t d = prim::block() * (uint32_t)kTapeThreads + tape_tid(); d < a.ndocs; d += stride) {
    const uint64_t w0 = ld64(a.dbase + 2 * (uint64_t)d), s0 = ld64(a.dbase + 2 * (uint64_t)d + 1);
    const uint64_t w1 = d + 1 < a.ndocs ? ld64(a.dbase + 2 * (uint64_t)d + 2) : tw;
    const uint64_t s1 = d + 1 < a.ndocs ? ld64(a.dbase + 2 * (uint64_t)d + 3) : ts;
    const uint64_t last = w1 - w0 - 1;
    st64(a.tape + w0, ((uint64_t)'r' << 56) | last);
    st64(a.tape + w0 + last, (uint64_t)'r' << 56);
    st64(a.out_pos + 4 * (uint64_t)d, w0);
    st64(a.out_pos + 4 * (uint64_t)d + 1, w1 - w0);
    st64(a.out_pos + 4 * (uint64_t)d + 2, s0);
    st64(a.out_pos + 4 * (uint64_t)d + 3, s1 - s0);
  }
}

// 4. Brackets and the strings' words; strings, numbers and literals queued
//    (one thread per entry, consecutive threads on consecutive entries; one
//    atomic per workgroup and queue).  In a batch, links and string offsets
//    are relative to the entry's document's tape and strings.
template <bool BATCH>
JSIDX_DEVFN void tape_write(const TapeArgs& a) {
  TapeChunkT<BATCH>& g = prim::lds_object<TapeChunkT<BATCH>>();
  const uint32_t tid = tape_tid();
  if (!batch_go<BATCH>(a)) return;
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  stage_offsets<BATCH>(a, n, g, tid, c);
  // the workgroup's slots in the two queues
  uint64_t cs = 0, cn = 0;
  for (int k = 0; k < kTapePer; k++) {
    const uint32_t j = (uint32_t)k * kTapeThreads + tid;
    const uint32_t b = g.K[j];  // entries past n were staged as ':'
    cs += b == '"';
    cn += words_of(b) == 2 || is_lit_start(b);  // numbers and literals share a queue
  }
  uint64_t sex, nex, sall, nall;
  group_scan2(g.sc, tid, cs, cn, &sex, &nex, &sall, &nall);
  if (tid == 0) {
    g.qbase[0] = sall ? prim::add_agent32(a.qcount + 1, (uint32_t)sall) : 0u;
    g.qbase[1] = nall ? prim::add_agent32(a.qcount + 2, (uint32_t)nall) : 0u;
  }
  prim::sync();
  uint32_t ps = g.qbase[0] + (uint32_t)sex, pn = g.qbase[1] + (uint32_t)nex;
  // a chunk's buffer bytes stay below 2^32 (its strings lie in the input,
  // fewer than 2^32 - 2^16 bytes), so an offset is the chunk base plus its
  // low word's distance from the base's
  const uint64_t sbase = ld64(a.chunk_sum + 2 * (uint64_t)c + 1);
  for (int k = 0; k < kTapePer; k++) {
    const uint32_t j = (uint32_t)k * kTapeThreads + tid;
    const uint64_t i = (uint64_t)c * kTapeChunk + j;
    if (i >= n) break;
    const uint32_t b = g.K[j];
    const uint64_t t = g.T[j];
    const bool bracket = b == '{' || b == '[' || b == '}' || b == ']';
    if (!bracket && b != '"' && !(words_of(b) == 2 || is_lit_start(b))) continue;
    uint32_t d = 0;
    uint64_t w0 = 0, s0 = 0;
    if (BATCH) {
      d = prim::load4(reinterpret_cast<const uint8_t*>(a.docid + i));
      w0 = ld64(a.dbase + 2 * (uint64_t)d);
      s0 = ld64(a.dbase + 2 * (uint64_t)d + 1);
    }
    if (bracket) {
      uint64_t link = 0;
      uint32_t m = kTapeUnlinked, lim = n, mv = 0;
      if (BATCH) {
        const uint32_t v0 = prim::load4(reinterpret_cast<const uint8_t*>(a.vstart + d));
        const uint64_t ob = prim::load8(a.offsets + d);
        m = prim::load4(reinterpret_cast<const uint8_t*>(a.match + ob + (i - v0)));
        lim = prim::load4(reinterpret_cast<const uint8_t*>(a.dn + d));
        mv = v0 + m;
      } else {
        m = prim::load4(reinterpret_cast<const uint8_t*>(a.match + i));
        mv = m;
      }
      if (m != kTapeUnlinked && m < lim) {
        const uint64_t tk = prim::load4(reinterpret_cast<const uint8_t*>(a.toff + mv)) - w0;
        link = (b == '{' || b == '[') ? tk + 1 : tk;
      }
      st64(a.tape + t, ((uint64_t)b << 56) | link);
    } else if (b == '"') {
      const uint64_t so = sbase + (uint32_t)(g.S[j] - (uint32_t)sbase);
      st64(a.tape + t, ((uint64_t)'"' << 56) | (so - s0));
      st64(a.squeue + 2 * (uint64_t)ps, i);
      st64(a.squeue + 2 * (uint64_t)ps + 1, so);
      ps++;
    } else {
      prim::st_out(a.nqueue + pn, (uint32_t)i);
      pn++;
    }
  }
  prim::sync();
  }
}

// Grid-stride bounds of a queue for this thread.
JSIDX_DEV uint32_t queue_len(const TapeArgs& a, int q) { return prim::ld_agent32(a.qcount + q); }

// 5. Strings: decoded into the buffer after their 32-bit length.
template <bool BATCH>
JSIDX_DEVFN void tape_strings(const TapeArgs& a) {
  if (!batch_go<BATCH>(a)) return;
  const uint32_t qn = queue_len(a, 1);
  const uint32_t stride = prim::grid() * (uint32_t)kTapeThreads;
  const uint32_t rounds = (qn + stride - 1) / stride;  // the same for every lane (wave_strings)
  for (uint32_t r = 0; r < rounds; r++) {
    const uint32_t q = r * stride + prim::block() * (uint32_t)kTapeThreads + tape_tid();
    const bool has = q < qn;
    uint64_t so = 0, pos = 0;
    uint32_t d = 0;
    if (has) {
      const uint32_t i = (uint32_t)ld64(a.squeue + 2 * (uint64_t)q);
      so = ld64(a.squeue + 2 * (uint64_t)q + 1);
      pos = entry_pos<BATCH>(a, i);
      d = entry_doc<BATCH>(a, i);
    }
    const TapeArgs la = entry_args<BATCH>(a, d);
    uint32_t k = 0;
    const uint32_t e = wave_strings<true>(la, has, pos, a.str + so + 4, &k);
    uint32_t err = 0;
    if (has) {
      err = e;
      for (int j = 0; j < 4; j++) prim::st_byte(a.str + so + j, (k >> (8 * j)) & 0xFFu);
    }
    or_flags<BATCH>(a, err, d);
  }
}

// 6. Numbers (both words; undecided doubles queued for tape_exact) and
//    literals.  (a: arguments whose bound is the entry's document; pos its
//    first byte.)
JSIDX_DEV uint32_t number_entry(const TapeArgs& a, uint64_t pos, uint64_t t, bool* undecided) {
  uint64_t* out = a.tape + t;
  *undecided = false;
  const uint32_t b = byte_at(a, pos);
  if (is_lit_start(b)) {  // a literal: its tag, and whether it is spelled out
    st64(out, (uint64_t)b << 56);
    return literal_ok(a, pos, b) ? 0u : kErrLiteral;
  }
  const NumText nt = scan_number(a, pos);
  if (!nt.ok) {
    st64(out, (uint64_t)'d' << 56);
    st64(out + 1, 0);
    return kErrNumber;
  }
  if (nt.is_int) {
    // at most 19 digits fit; the magnitude limit is 2^63 - 1, or 2^63 if negative
    const uint64_t lim = nt.neg ? (1ull << 63) : (1ull << 63) - 1u;
    st64(out, (uint64_t)'l' << 56);
    if (nt.int_digits > 19 || nt.w > lim) {
      st64(out + 1, 0);
      return kErrNumber;
    }
    st64(out + 1, nt.neg ? 0ull - nt.w : nt.w);
    return 0;
  }
  st64(out, (uint64_t)'d' << 56);
  const uint64_t sign = nt.neg ? 1ull << 63 : 0ull;
  if (nt.w == 0) {
    st64(out + 1, sign);
    return 0;
  }
  uint64_t bits = 0;
  int r = fast_double(nt.w, nt.q, &bits);
  if (r != kConvUndecided && nt.trunc) {
    // the value lies strictly between w and w + 1 (times 10^q): decided only
    // if both ends give the same result
    uint64_t bits2 = 0;
    const int r2 = fast_double(nt.w + 1, nt.q, &bits2);
    if (r2 != r || (r == kConvOk && bits2 != bits)) r = kConvUndecided;
  }
  if (r == kConvInf) {
    st64(out + 1, 0);
    return kErrNumber;
  }
  if (r == kConvUndecided) {
    *undecided = true;
    return 0;
  }
  st64(out + 1, bits | sign);
  return 0;
}

template <bool BATCH>
JSIDX_DEVFN void tape_numbers(const TapeArgs& a) {
  if (!batch_go<BATCH>(a)) return;
  const uint32_t qn = queue_len(a, 2);
  const uint32_t stride = prim::grid() * (uint32_t)kTapeThreads;
  const uint32_t rounds = (qn + stride - 1) / stride;
  for (uint32_t r = 0; r < rounds; r++) {
    const uint32_t q = r * stride + prim::block() * (uint32_t)kTapeThreads + tape_tid();
    bool undecided = false;
    uint32_t i = 0, d = 0, err = 0;
    if (q < qn) {
      i = prim::load4(reinterpret_cast<const uint8_t*>(a.nqueue + q));
      d = entry_doc<BATCH>(a, i);
      const uint64_t t = prim::load4(reinterpret_cast<const uint8_t*>(a.toff + i));
      err = number_entry(entry_args<BATCH>(a, d), entry_pos<BATCH>(a, i), t, &undecided);
    }
    const uint32_t slot = wave_append(a, 0, undecided);
    if (undecided) prim::st_out(a.queue + slot, i);
    or_flags<BATCH>(a, err, d);
  }
}

// 7. The queued numbers, one thread each, by exact arithmetic.
struct ExactScratch {
  Big D, V, S;
};

template <bool BATCH>
JSIDX_DEV void exact_entry(const TapeArgs& a, uint32_t i, ExactScratch& x) {
  const uint32_t d = entry_doc<BATCH>(a, i);
  const TapeArgs la = entry_args<BATCH>(a, d);
  const uint64_t pos = entry_pos<BATCH>(a, i);
  const uint64_t t = prim::load4(reinterpret_cast<const uint8_t*>(a.toff + i));
  uint64_t bits = 0;
  const int r = exact_double(la, pos, x.D, x.V, x.S, &bits);
  if (r == kConvInf) {
    st64(a.tape + t + 1, 0);
    prim::or_agent32(a.err + d, kErrNumber);
    return;
  }
  const uint64_t sign = byte_at(la, pos) == '-' ? 1ull << 63 : 0ull;
  st64(a.tape + t + 1, bits | sign);
}

template <bool BATCH>
JSIDX_DEVFN void tape_exact(const TapeArgs& a) {
  if (!batch_go<BATCH>(a)) return;
  ExactScratch x;
  const uint32_t qn = prim::ld_agent32(a.qcount);
  const uint32_t stride = prim::grid() * (uint32_t)kExactThreads;
  for (uint32_t q = prim::block() * (uint32_t)kExactThreads + prim::lane(); q < qn; q += stride)
    exact_entry<BATCH>(a, prim::load4(reinterpret_cast<const uint8_t*>(a.queue + q)), x);
}

// ---- Batches ---------------------------------------------------------------
// 0. The first virtual entry of each document (an empty document counts one
//    placeholder entry): sums per 2048 documents (tape_batch_sums), the sums
//    scanned with the totals and the queues emptied (tape_batch_bases, one
//    workgroup), every document's start and cleared flags
//    (tape_batch_starts).  A batch with more virtual entries than the
//    workspace holds, or whose bytes reach 2^32 - 2^16, is not written:
//    every document gets JSIDX_ERR_CAPACITY and the kernels after these do
//    nothing.
JSIDX_DEVFN void tape_batch_sums(const TapeArgs& a) { docscan_sums(a.dn, a.ndocs, true, a.part); }

JSIDX_DEVFN void tape_batch_bases(const TapeArgs& a) {
  const uint64_t total = docscan_bases((uint32_t)docscan_groups(a.ndocs), a.part);
  if (tape_tid() == 0) {
    const uint64_t span = prim::load8(a.offsets + a.ndocs) - prim::load8(a.offsets);
    const bool over = total > (uint64_t)a.cap || span >= (1ull << 32) - (1ull << 16);
    if (!over) prim::st_out(a.vstart + a.ndocs, (uint32_t)total);
    prim::st_out(a.vn, over ? 0u : (uint32_t)total);
    prim::st_out(a.vn + 1, over ? 0u : (uint32_t)((total + kTapeChunk - 1) / kTapeChunk));
    prim::st_out(a.vn + 2, 0u);
    prim::st_out(a.vn + 3, over ? 1u : 0u);
    for (int q = 0; q < 3; q++) prim::st_out(a.qcount + q, 0u);
  }
}

JSIDX_DEVFN void tape_batch_starts(const TapeArgs& a) {
  const bool over = prim::ld_agent32(a.vn + 3) != 0u;
  docscan_starts(a.dn, a.ndocs, true, a.part, [&](uint64_t d, uint64_t start, uint32_t) {
    if (!over) prim::st_out(a.vstart + d, (uint32_t)start);
    prim::st_out(a.err + d, over ? kTapeErrCapacity : 0u);
  });
}

// 1b. Each document's entries into the virtual sequence: absolute positions,
//     document numbers and flags (one wave per document).
JSIDX_DEVFN void tape_batch_compact(const TapeArgs& a) {
  const uint32_t lane = prim::lane();
  if (prim::ld_agent32(a.vn + 1) == 0u) return;
  const uint32_t waves_per_group = kTapeThreads / 64u;
  const uint32_t nw = prim::grid() * waves_per_group;
  for (uint32_t d = prim::block() * waves_per_group + prim::wave_id(); d < a.ndocs; d += nw) {
    const uint64_t base = prim::load8(a.offsets + d);
    const uint32_t nd = prim::load4(reinterpret_cast<const uint8_t*>(a.dn + d));
    const uint32_t v0 = prim::load4(reinterpret_cast<const uint8_t*>(a.vstart + d));
    const uint32_t cnt = nd ? nd : 1u;
    for (uint32_t j = lane; j < cnt; j += 64u) {
      uint32_t f = 0;
      uint64_t pos = base;
      if (nd) pos += prim::load4(reinterpret_cast<const uint8_t*>(a.idx + base + j));
      else f |= kVEmpty;
      if (j == 0) f |= kVFirst;
      if (j + 1 == cnt) f |= kVLast;
      st64(a.vpos + v0 + j, pos);
      prim::st_byte(a.vflag + v0 + j, f);
      prim::st_out(a.docid + v0 + j, d);
    }
  }
}

}  // namespace jsidx
