// jsidx_tape.h -- stage 2's tape (Sec. 3, Fig. 2) from a document's structural
// index and scope links: 64-bit words tagged with a character in bits 56..63,
// numbers parsed (two words: 'l' and an int64, or 'd' and a binary64), strings
// normalized into a string buffer (a 32-bit length, then UTF-8), literals
// checked.  Once the index is known no token depends on another (Sec. 3.2), so
// every entry is handled by its own thread:
//   1. tape_count: each entry's first byte and the buffer bytes of each string
//      (decoded, not written) go to the workspace; the words (0 for ':' and
//      ',', 2 for a number, else 1) and bytes are summed per chunk of 2048
//      entries;
//   2. tape_scan: one workgroup turns the chunk sums into bases and writes the
//      root words, the sizes, and clears the flags;
//   3. tape_offsets: each bracket's tape index (a scan inside the chunk);
//   4. tape_write: the words of brackets (with the tape index of their
//      partner, from the scope links) and strings; strings decoded into the
//      buffer; numbers with literals queued densely, each with its tape
//      index (and its first byte's position where the pass has it), for
//   5. tape_numbers: literals checked, numbers converted; a double whose
//      rounding the fast conversion cannot decide is queued again for
//   6. tape_exact: the exact big-integer conversion.
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
constexpr int kTapePer = 8;
constexpr int kTapeChunk = kTapeThreads * kTapePer;
constexpr int kTapeSuper = 4;  // groups of 64 entries in a run (below)
static_assert(kTapePer % kTapeSuper == 0, "a wave's entries are whole runs");
constexpr uint32_t kRunMax = 64u * kTapeSuper;  // entries of a run
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
  uint8_t* runbad;      // per run of kRunMax entries: 1 if its strings take the per-string path
  uint32_t* toff;       // per entry: tape index of its first word (brackets only)
  uint32_t* qcount;     // queue lengths: [0] exact conversions, [1] numbers, [2] literals
  uint32_t* queue;      // number-queue slots for the exact conversion
  uint2* nqueue;        // numbers (from the front) and literals (from the back): the
                        // first byte's position or the entry (queue_key), and the
                        // tape index
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
  uint64_t vn, tot, qcount, part, vstart, docid, vpos, vflag, dbase, chunk_sum, sbytes, kb, runbad, toff, queue,
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
  L.runbad = o; o = al(o + cap / kRunMax + 1);
  L.toff = o; o = al(o + cap * 4);
  L.queue = o; o = al(o + cap * 4);
  L.nqueue = o; o = al(o + cap * 8);
  L.total = o;
  return L;
}

struct TapeLayout {
  uint64_t chunk_sum, sbytes, kb, runbad, toff, qcount, queue, nqueue, total;
};
inline uint64_t tape_align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }
inline TapeLayout tape_layout(uint64_t n) {
  const uint64_t nc = (n + kTapeChunk - 1) / kTapeChunk;
  TapeLayout L;
  uint64_t o = 0;
  L.chunk_sum = o; o = tape_align256(o + nc * 16);
  L.sbytes = o; o = tape_align256(o + n * 4);
  L.kb = o; o = tape_align256(o + n);
  L.runbad = o; o = tape_align256(o + n / kRunMax + 1);
  L.toff = o; o = tape_align256(o + n * 4);
  L.qcount = o; o = tape_align256(o + 16);
  L.queue = o; o = tape_align256(o + n * 4);
  L.nqueue = o; o = tape_align256(o + n * 8);
  L.total = o;
  return L;
}

JSIDX_DEV uint32_t tape_tid() { return prim::wave_id() * 64u + prim::lane(); }

JSIDX_DEV uint32_t byte_at(const TapeArgs& a, uint64_t p) { return p < a.len ? prim::load1(a.buf + p) : 0u; }

// The first byte of entry i (0 if its position is not inside the document).
JSIDX_DEV uint32_t entry_byte(const TapeArgs& a, uint32_t i) {
  return byte_at(a, prim::load4(reinterpret_cast<const uint8_t*>(a.idx + i)));
}

// Sets of first bytes as two 64-bit masks (bytes 0..63, 64..127), tested
// without branches: chains of comparisons become branches and mask
// arithmetic in divergent code.
constexpr uint64_t set_lo(uint32_t c) { return c < 64 ? 1ull << c : 0ull; }
constexpr uint64_t set_hi(uint32_t c) { return c >= 64 && c < 128 ? 1ull << (c - 64) : 0ull; }
JSIDX_DEV bool in_set(uint32_t b, uint64_t lo, uint64_t hi) {
  const uint64_t m = (b & 64u) ? hi : lo;
  return ((uint32_t)(m >> (b & 63u)) & (b < 128u ? 1u : 0u)) != 0u;
}
constexpr uint64_t kLitHi = set_hi('t') | set_hi('f') | set_hi('n');
constexpr uint64_t kBracketHi = set_hi('{') | set_hi('}') | set_hi('[') | set_hi(']');
constexpr uint64_t kNoWordLo = set_lo(':') | set_lo(',');
JSIDX_DEV bool is_lit_start(uint32_t b) { return in_set(b, 0u, kLitHi); }
JSIDX_DEV bool is_bracket(uint32_t b) { return in_set(b, 0u, kBracketHi); }

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
  // none for ':' and ',', one for brackets, strings and literals, else two
  // (a number, or an invalid atom, which is a number error)
  const bool none = in_set(b, kNoWordLo, 0u), one = in_set(b, set_lo('"'), kBracketHi | kLitHi);
  return 2u - (none ? 2u : 0u) - (one ? 1u : 0u);
}

// An atom ends at white space, a structural character or the document's end.
JSIDX_DEV bool ends_atom(const Window& w, uint64_t p) {
  if (p >= w.len) return true;
  const uint32_t c = win_byte(w, p);
  return c == ' ' || c == '\t' || c == '\n' || c == '\r' || c == ',' || c == ':' || c == '[' || c == ']' ||
         c == '{' || c == '}';
}

// ---- Strings (Sec. 3.2.2) ---------------------------------------------------
// The string passes take the entries 64 at a time, one per lane of a wave.
// The wave first copies the document bytes of its group (from the group's
// first entry, or first string, up to the entry after the group: every
// string of the group lies there) into LDS with 16-byte loads, consecutive
// lanes on consecutive blocks, so that the document is read once and
// coalesced; each lane then scans its own string there, 16 bytes per step.
// Bytes past the copy (a group longer than kStrIn bytes) are read from the
// document itself.  The writing pass also stages the group's output (each
// string's length word and bytes, contiguous in the buffer) in LDS and
// stores it with 16-byte stores; a string whose output does not fit there
// is written to the buffer directly.
constexpr uint32_t kStrIn = 2048;   // staged document bytes per wave
constexpr uint32_t kStrOut = 2048;  // staged buffer bytes per wave
struct alignas(16) StrLds {
  uint32_t in[kStrIn / 4];
  uint32_t out[kStrOut / 4];
};

// Where a lane reads its string: the document (its bytes below len belong to
// the entry's document; 16-byte loads start at or after blo) and the wave's
// copy of positions [lo, hi) (lo 16-byte aligned as an address; hi == lo:
// nothing staged).
struct StrSrc {
  const uint8_t* buf;
  uint64_t len;
  uint64_t blo;
  uint64_t lo, hi;
};

// Word k (0..3) of four, by mask arithmetic (a runtime index, or a chain of
// selects the compiler may turn into one, would put the words in private
// memory).
JSIDX_DEV uint32_t word_in(const uint32_t x[4], uint32_t k) {
  return (x[0] & (0u - (uint32_t)(k == 0))) | (x[1] & (0u - (uint32_t)(k == 1))) |
         (x[2] & (0u - (uint32_t)(k == 2))) | (x[3] & (0u - (uint32_t)(k == 3)));
}

// Byte p (p < len).
JSIDX_DEV uint32_t src_byte(const StrSrc& s, const StrLds& L, uint64_t p) {
  if (p >= s.lo && p < s.hi) return prim::lds_ld1(reinterpret_cast<const uint8_t*>(L.in) + (p - s.lo));
  return prim::load1(s.buf + p);
}

// The 16-byte aligned block holding byte p, if all of it lies inside the
// entry's document: its words in x, its first position returned (else ~0).
JSIDX_DEV uint64_t src_block(const StrSrc& s, const StrLds& L, uint64_t p, uint32_t x[4]) {
  const uint64_t off = reinterpret_cast<uintptr_t>(s.buf + p) & 15u;
  if (p < s.blo + off || p - off + 16 > s.len) return ~0ull;
  const uint64_t pb = p - off;
  const uint4 v = pb >= s.lo && pb + 16 <= s.hi ? prim::ld_lds128(L.in + (pb - s.lo) / 4) : prim::load16(s.buf + pb);
  x[0] = v.x;
  x[1] = v.y;
  x[2] = v.z;
  x[3] = v.w;
  return pb;
}

// Copies positions [lo, hi) of buf into L.in (whole wave; 16-byte loads
// where the block lies inside [blo, bhi), bytes at the buffer's ends) and
// returns the staged end (hi rounded up to the block, within bhi).
JSIDX_DEV uint64_t stage_in(StrLds& L, const uint8_t* buf, uint64_t lo, uint64_t hi, uint64_t bhi) {
  const uint32_t nblk = (uint32_t)((hi - lo + 15) / 16);
  for (uint32_t m = prim::lane(); m < nblk; m += 64u) {
    const uint64_t pb = lo + 16ull * m;
    uint4 v;
    if (pb + 16 <= bhi) {
      v = prim::load16(buf + pb);
    } else {
      uint32_t w[4] = {0u, 0u, 0u, 0u};
      for (uint32_t b = 0; b < 16u; b++)
        if (pb + b < bhi) w[b / 4] |= prim::load1(buf + pb + b) << (8 * (b % 4));
      v = uint4{w[0], w[1], w[2], w[3]};
    }
    prim::st_lds128(L.in + 4 * m, v);
  }
  const uint64_t end = lo + 16ull * nblk;
  return end < bhi ? end : bhi;
}

// Stages the bytes of a group that start at p0 (its first entry or string)
// and end before p1 (the entry after the group, or the buffer's end), at most
// kStrIn of them, for the lanes' reads (whole wave; the range is the same
// for every lane).  [blo, bhi) is the readable buffer.
JSIDX_DEV StrSrc stage_group(StrLds& L, const uint8_t* buf, uint64_t p0, uint64_t p1, uint64_t blo, uint64_t bhi) {
  StrSrc s{buf, 0, blo, 0, 0};
  const uint64_t off = reinterpret_cast<uintptr_t>(buf + p0) & 15u;
  uint64_t lo = p0 - off;
  if (p0 < blo + off) lo = p0 + ((16u - off) & 15u);  // the buffer's first bytes stay in memory
  uint64_t hi = p1 > lo ? p1 : lo;
  if (hi > lo + kStrIn) hi = lo + kStrIn;
  if (hi > bhi) hi = bhi > lo ? bhi : lo;
  prim::wave_sync();  // the previous group's reads are done
  s.lo = lo;
  s.hi = stage_in(L, buf, lo, hi, bhi);
  prim::wave_sync();
  return s;
}

// Where a lane writes its string's bytes: the buffer at g, or (staged) the
// wave's output copy at L.out byte li, which has g's alignment.
struct StrDst {
  uint8_t* g;
  uint32_t li;
  bool staged;
};
JSIDX_DEV void dst_byte(const StrDst& o, StrLds& L, uint32_t k, uint32_t v) {
  if (!o.staged) {
    prim::st_byte(o.g + k, v);
  } else if (o.li + k < kStrOut) {  // always (the count pass sized the string)
    prim::lds_st1(reinterpret_cast<uint8_t*>(L.out) + o.li + k, v);
  }
}
// A word to a 4-byte aligned destination.
JSIDX_DEV void dst_word(const StrDst& o, StrLds& L, uint32_t k, uint32_t v) {
  if (!o.staged) {
    prim::st_out(reinterpret_cast<uint32_t*>(o.g + k), v);
  } else if (o.li + k + 4 <= kStrOut) {
    prim::lds_st4(L.out + (o.li + k) / 4, v);
  }
}

JSIDX_DEV int32_t hex_digit(uint32_t c) {
  if (c >= '0' && c <= '9') return (int32_t)(c - '0');
  if (c >= 'a' && c <= 'f') return (int32_t)(c - 'a' + 10);
  if (c >= 'A' && c <= 'F') return (int32_t)(c - 'A' + 10);
  return -1;
}

// Four hex digits at p, or -1.
JSIDX_DEV int32_t hex_quad(const StrSrc& s, const StrLds& L, uint64_t p) {
  if (p + 4 > s.len) return -1;
  int32_t v = 0;
  for (int k = 0; k < 4; k++) {
    const int32_t h = hex_digit(src_byte(s, L, p + k));
    if (h < 0) return -1;
    v = v * 16 + h;
  }
  return v;
}

constexpr uint32_t kDeferred = 0x80000000u;  // string_run: the budget ran out

// The escape whose backslash is at *p: its bytes (\uXXXX and surrogate pairs
// as UTF-8) written if `writer`, *p and *k past it.  Returns 0 or kErrString.
template <bool WRITE>
JSIDX_DEV uint32_t escape_at(const StrSrc& s, StrLds& L, uint64_t* pp, const StrDst& o, uint32_t* kk, bool writer) {
  uint64_t p = *pp;
  uint32_t k = *kk;
  auto put = [&](uint32_t v) {
    if constexpr (WRITE) {
      if (writer) dst_byte(o, L, k, v);
    }
    k++;
  };
  if (p + 1 >= s.len) return kErrString;
  const uint32_t e = src_byte(s, L, p + 1);
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
    const int32_t u = hex_quad(s, L, p);
    if (u < 0) return kErrString;
    p += 4;
    uint32_t cp = (uint32_t)u;
    if (cp >= 0xDC00u && cp <= 0xDFFFu) return kErrString;  // a low surrogate first
    if (cp >= 0xD800u && cp <= 0xDBFFu) {
      if (p + 2 > s.len || src_byte(s, L, p) != '\\' || src_byte(s, L, p + 1) != 'u') return kErrString;
      const int32_t lo = hex_quad(s, L, p + 2);
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

// Bytes [off, first) of a 16-byte block (words x) to the destination at k:
// single bytes up to a 4-byte aligned destination, whole words taken from
// the block shifted as a 128-bit value, single bytes after them.
JSIDX_DEV void copy_plain(const StrDst& o, StrLds& L, uint32_t k, const uint32_t x[4], uint32_t off, uint32_t first) {
  const uint64_t lo64 = ((uint64_t)x[1] << 32) | x[0], hi64 = ((uint64_t)x[3] << 32) | x[2];
  const uint32_t cnt = first - off;
  const uint32_t da = (uint32_t)(reinterpret_cast<uintptr_t>(o.g + k) & 3u);
  uint32_t m0 = (4u - da) & 3u;
  if (m0 > cnt) m0 = cnt;
  const uint32_t nw = (cnt - m0) / 4;
  for (uint32_t m = 0; m < cnt; m++) {
    if (m == m0 && nw) m += 4 * nw;  // the words below
    if (m >= cnt) break;
    const uint32_t idx = off + m;
    dst_byte(o, L, k + m, (uint32_t)((idx < 8 ? lo64 >> (8 * idx) : hi64 >> (8 * (idx - 8))) & 0xFFu));
  }
  if (nw) {
    const uint32_t r = 8 * (off + m0);  // at most 96: off + m0 + 4 <= first <= 16
    const uint64_t slo = r == 0 ? lo64 : r < 64 ? (lo64 >> r) | (hi64 << (64 - r)) : hi64 >> (r - 64);
    const uint64_t shi = r < 64 ? hi64 >> r : 0ull;
    dst_word(o, L, k + m0, (uint32_t)slo);
    if (nw > 1) dst_word(o, L, k + m0 + 4, (uint32_t)(slo >> 32));
    if (nw > 2) dst_word(o, L, k + m0 + 8, (uint32_t)shi);
    if (nw > 3) dst_word(o, L, k + m0 + 12, (uint32_t)(shi >> 32));
  }
}

// One lane's part of a string: from byte *p on (inside the string, *k bytes
// already out) up to the closing quote, in at most `budget` steps (a block
// of plain bytes, or one escape or single byte each).  Returns 0 (closed),
// kErrString (a byte below 0x20, a bad escape, no closing quote; the count
// then stops there, the same in both passes) or kDeferred (*p and *k say
// where it stopped).
template <bool WRITE>
JSIDX_DEV uint32_t string_run(const StrSrc& s, StrLds& L, uint64_t* pp, const StrDst& o, uint32_t* kk,
                              uint32_t budget) {
  uint64_t p = *pp;
  uint32_t k = *kk;
  uint32_t err = 0;
  uint32_t steps = 0;
  for (;;) {
    // the aligned block holding p: the plain bytes up to the first quote,
    // backslash or control byte are taken from registers; that byte is
    // handled below
    uint32_t x[4];
    const uint64_t pb = src_block(s, L, p, x);
    if (pb != ~0ull) {
      const uint32_t off = (uint32_t)(p - pb);
      // the lowest flagged byte of a word is exact (a borrow only runs upward)
      auto hits = [](uint32_t v) {
        const uint32_t q2 = v ^ 0x22222222u, b2 = v ^ 0x5C5C5C5Cu;
        return (((q2 - 0x01010101u) & ~q2) | ((b2 - 0x01010101u) & ~b2) | ((v - 0x20202020u) & ~v)) & 0x80808080u;
      };
      // bytes of word j at or after p
      auto keep = [off](uint32_t j) {
        return off <= 4 * j ? 0xFFFFFFFFu : off >= 4 * j + 4 ? 0u : 0xFFFFFFFFu << (8 * (off - 4 * j));
      };
      const uint32_t h0 = hits(x[0]) & keep(0), h1 = hits(x[1]) & keep(1);
      const uint32_t h2 = hits(x[2]) & keep(2), h3 = hits(x[3]) & keep(3);
      // the first special byte at or after p, in the block (16: none)
      const uint32_t first = h0 ? (uint32_t)__builtin_ctz(h0) / 8
                           : h1 ? 4 + (uint32_t)__builtin_ctz(h1) / 8
                           : h2 ? 8 + (uint32_t)__builtin_ctz(h2) / 8
                           : h3 ? 12 + (uint32_t)__builtin_ctz(h3) / 8 : 16u;
      if constexpr (WRITE) copy_plain(o, L, k, x, off, first);
      k += first - off;
      p = pb + first;
      if (first == 16) {
        if (++steps >= budget) { err = kDeferred; break; }
        continue;
      }
      // the special byte is in the registers: a closing quote ends the string
      // without another load
      if (((word_in(x, first / 4) >> (8 * (first & 3u))) & 0xFFu) == '"') break;
    }
    if (p >= s.len) { err = kErrString; break; }
    const uint32_t c = src_byte(s, L, p);
    if (c == '"') break;
    if (c < 0x20u) { err = kErrString; break; }
    if (c != '\\') {
      if constexpr (WRITE) dst_byte(o, L, k, c);
      k++;
      p++;
    } else {
      err = escape_at<WRITE>(s, L, &p, o, &k, true);
      if (err) break;
    }
    if (++steps >= budget) { err = kDeferred; break; }
  }
  *pp = p;
  *kk = k;
  return err;
}

JSIDX_DEV uint64_t readlane64(uint64_t v, int l) {
  return ((uint64_t)prim::readlane((uint32_t)(v >> 32), l) << 32) | prim::readlane((uint32_t)v, l);
}

// UTF-8 of code point cp: its bytes, lowest first, in one word; *n their count.
JSIDX_DEV uint32_t utf8_of(uint32_t cp, uint32_t* n) {
  if (cp < 0x80u) { *n = 1; return cp; }
  if (cp < 0x800u) { *n = 2; return (0xC0u | (cp >> 6)) | ((0x80u | (cp & 0x3Fu)) << 8); }
  if (cp < 0x10000u) {
    *n = 3;
    return (0xE0u | (cp >> 12)) | ((0x80u | ((cp >> 6) & 0x3Fu)) << 8) | ((0x80u | (cp & 0x3Fu)) << 16);
  }
  *n = 4;
  return (0xF0u | (cp >> 18)) | ((0x80u | ((cp >> 12) & 0x3Fu)) << 8) | ((0x80u | ((cp >> 6) & 0x3Fu)) << 16) |
         ((0x80u | (cp & 0x3Fu)) << 24);
}

// The byte an escape letter stands for (0x100: not an escape letter; 'u' is
// handled apart).
JSIDX_DEV uint32_t escape_char(uint32_t e) {
  switch (e) {
    case '"': return '"';
    case '\\': return '\\';
    case '/': return '/';
    case 'b': return 0x08u;
    case 'f': return 0x0Cu;
    case 'n': return 0x0Au;
    case 'r': return 0x0Du;
    case 't': return 0x09u;
    default: return 0x100u;
  }
}

// 64 bytes of a string from p on (p not inside an escape) by the whole wave,
// one byte per lane, every escape in them decoded at once (every lane calls
// it with the same arguments).  The escapes are found from the backslash
// mask: the lowest backslash left starts one, which covers the byte after it
// (scalar work, a few steps per window).  The window ends at the closing
// quote, or before an escape that runs past its 64 bytes.  Returns the bytes
// taken (*closed: up to the closing quote) after writing their decoded bytes
// at *k (prefix sum of each lane's byte count), or -1 without writing if the
// bytes taken would hold a byte below 0x20, a bad escape or a bad \u
// sequence, or run past the document (the serial step then takes them, with
// its error rules).
template <bool WRITE>
JSIDX_DEV int string_window(const StrSrc& s, StrLds& L, uint64_t p, const StrDst& o, uint32_t* kk, bool* closed) {
  const uint32_t lane = prim::lane();
  const uint64_t pos = p + lane;
  const uint32_t c = pos < s.len ? src_byte(s, L, pos) : 0x100u;
  const uint64_t bsl = prim::ballot(c == '\\'), quo = prim::ballot(c == '"');
  const uint64_t ctl = prim::ballot(c < 0x20u || c >= 0x100u);
  uint64_t esc = 0, st = 0, rem = bsl;  // escaped bytes, escape-starting backslashes
  while (rem) {
    const int i = __builtin_ctzll(rem);
    st |= 1ull << i;
    if (i == 63) break;
    esc |= 2ull << i;
    rem &= i == 62 ? 0ull : ~((4ull << i) - 1);
  }
  const bool is_esc = prim::lane_bit(esc), is_st = prim::lane_bit(st);
  // \u escapes: the letter's lane reads the four hex digits (and those of a
  // low surrogate after a high one)
  const bool is_u = is_esc && c == 'u';
  int32_t cp = -1;
  bool pair = false;
  if (is_u) {
    cp = hex_quad(s, L, pos + 1);
    if (cp >= 0xD800 && cp <= 0xDBFF) {
      const int32_t lo = pos + 6 < s.len && src_byte(s, L, pos + 5) == '\\' && src_byte(s, L, pos + 6) == 'u'
                             ? hex_quad(s, L, pos + 7) : -1;
      if (lo >= 0xDC00 && lo <= 0xDFFF) {
        cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
        pair = true;
      } else {
        cp = -1;
      }
    } else if (cp >= 0xDC00 && cp <= 0xDFFF) {
      cp = -1;
    }
  }
  const uint64_t um = prim::ballot(is_u), pm = prim::ballot(pair);
  const uint64_t hex = (um << 1) | (um << 2) | (um << 3) | (um << 4) | (pm << 5) | (pm << 6);  // the pair's
  // second backslash is in st already; its letter and digits are covered by
  // pm << 6 and um's own shifts (the second letter is escaped too)
  const uint64_t second = pm << 6;
  // the closing quote, and the first escape whose bytes do not all lie in the window
  const uint64_t endq = quo & ~esc & ~hex;
  const uint32_t end = endq ? (uint32_t)__builtin_ctzll(endq) : 64u;
  const uint32_t seq = prim::lane_bit(um >> 1) ? (prim::lane_bit(pm >> 1) ? 12u : 6u) : 2u;
  const uint64_t over = prim::ballot(is_st && lane + seq > 64u);
  const uint32_t cut = over ? (uint32_t)__builtin_ctzll(over) : 64u;
  const uint32_t W = end < cut ? end : cut;
  const uint64_t take = W >= 64 ? ~0ull : (1ull << W) - 1;
  // anything the fast path does not decode
  const bool bad_here = (is_esc && !(second >> lane & 1ull) && (c == 'u' ? cp < 0 : escape_char(c) == 0x100u));
  const uint64_t bad = (ctl | prim::ballot(bad_here)) & take & ~(hex & ~second);
  if (bad) return -1;
  // each lane's bytes
  uint32_t n = 0, v = 0;
  if (lane < W && !is_st && !(hex >> lane & 1ull)) {
    if (is_u) v = utf8_of((uint32_t)cp, &n);
    else if (is_esc) { v = escape_char(c); n = 1; }
    else { v = c; n = 1; }
  }
  const uint32_t incl = prim::incl_scan(n);
  uint32_t k = *kk;
  if constexpr (WRITE) {
    for (uint32_t j = 0; j < n; j++) dst_byte(o, L, k + incl - n + j, (v >> (8 * j)) & 0xFFu);
  }
  k += prim::readlane(incl, 63);
  *kk = k;
  *closed = end < cut;
  return (int)W;
}

// The rest of a string by the whole wave (every lane calls it with the same
// arguments): 64 bytes per step (string_window); a window holding an error
// candidate is taken serially instead: its plain bytes up to the first quote,
// backslash or control byte, found by ballot, written by their lanes, then
// that byte (an escape is decoded by every lane and written by lane 0).
// Returns 0 or kErrString; *k as string_run.
template <bool WRITE>
JSIDX_DEV uint32_t string_wave(const StrSrc& s, StrLds& L, uint64_t p, const StrDst& o, uint32_t* kk) {
  const uint32_t lane = prim::lane();
  uint32_t k = *kk;
  uint32_t err = 0;
  for (;;) {
    bool closed = false;
    const int w = string_window<WRITE>(s, L, p, o, &k, &closed);
    if (w >= 0) {
      p += (uint32_t)w;
      if (closed) break;
      continue;
    }
    const uint64_t pos = p + lane;
    const uint32_t c = pos < s.len ? src_byte(s, L, pos) : 0x100u;
    const bool special = c >= 0x100u || c == '"' || c == '\\' || c < 0x20u;
    const uint64_t m = prim::ballot(special);
    const uint32_t f = m ? (uint32_t)__builtin_ctzll(m) : 64u;
    if constexpr (WRITE) {
      if (lane < f) dst_byte(o, L, k + lane, c);
    }
    k += f;
    p += f;
    if (f == 64) continue;
    const uint32_t c0 = prim::readlane(c, (int)f);  // the special byte, the same for every lane
    if (c0 == '"') break;
    if (c0 >= 0x100u || c0 < 0x20u) { err = kErrString; break; }
    err = escape_at<WRITE>(s, L, &p, o, &k, lane == 0);
    if (err) break;
  }
  *kk = k;
  return err;
}


// Strings of a wave, each lane's string opening at q (if `has`): its bytes
// after normalization (escapes decoded, \uXXXX and surrogate pairs as UTF-8)
// to o (WRITE) and their count to *n.  A byte below 0x20, an unknown escape,
// a malformed or lone surrogate, or no closing quote is an error (the count
// then stops there, the same in both passes).  Each lane runs its own string
// for kStringSteps steps; the strings that outrun it are then finished one
// after another by the whole wave.  Every lane of the wave must call this.
constexpr uint32_t kStringSteps = 3;
template <bool WRITE>
JSIDX_DEV uint32_t wave_strings(const StrSrc& s, StrLds& L, bool has, uint64_t q, const StrDst& o, uint32_t* n) {
  uint64_t p = q + 1;
  uint32_t k = 0;
  uint32_t err = has ? string_run<WRITE>(s, L, &p, o, &k, kStringSteps) : 0u;
  uint64_t m = prim::ballot(err == kDeferred);
  while (m) {
    const int l = __builtin_ctzll(m);
    m &= m - 1;
    const uint64_t pl = readlane64(p, l);
    uint32_t kl = prim::readlane(k, l);
    // the lane's own document bound and destination
    StrSrc sl = s;
    sl.len = readlane64(s.len, l);
    StrDst ol{nullptr, 0u, false};
    if constexpr (WRITE) {
      ol.g = reinterpret_cast<uint8_t*>(readlane64(reinterpret_cast<uintptr_t>(o.g), l));
      ol.li = prim::readlane(o.li, l);
      ol.staged = prim::readlane(o.staged ? 1u : 0u, l) != 0u;
    }
    const uint32_t e = string_wave<WRITE>(sl, L, pl, ol, &kl);
    if ((int)prim::lane() == l) {
      k = kl;
      err = e;
    }
  }
  *n = k;
  return err;
}

// Stores a wave's staged output: buffer bytes [A, B), staged from L.out byte
// d on (d: A's offset in its 16-byte block); whole blocks with 16-byte
// stores, the partial blocks at both ends byte by byte (whole wave).
JSIDX_DEV void copy_out(StrLds& L, uint8_t* str, uint64_t A, uint64_t B, uint32_t d) {
  prim::wave_sync();  // every lane's staged bytes are written
  const uint32_t end = (uint32_t)(B - A) + d;  // staged bytes [d, end)
  const uint32_t nblk = (end + 15) / 16;
  for (uint32_t m = prim::lane(); m < nblk; m += 64u) {
    const uint32_t u0 = 16 * m;
    if (u0 >= d && u0 + 16 <= end) {
      prim::st_out4(reinterpret_cast<uint32_t*>(str + (A + (u0 - d))), prim::ld_lds128(L.out + 4 * m));
    } else {
      for (uint32_t b = 0; b < 16u; b++) {
        const uint32_t u = u0 + b;
        if (u >= d && u < end)
          prim::st_byte(str + (A + (u - d)), prim::lds_ld1(reinterpret_cast<const uint8_t*>(L.out) + u));
      }
    }
  }
}

// ---- Strings, byte-parallel ---------------------------------------------------
// The fast path of a run of kRunMax entries: the bytes from its first string
// on are taken 1 KiB per step, lane l holding bytes 16 l .. 16 l + 15 of the
// step (one 16-byte load), and every byte is classified at once (quote,
// backslash, byte below 0x20) by word arithmetic.  What a byte is follows
// from masks and from carries between lanes and steps:
//  - the escapes: the lowest backslash not yet covered starts one, which
//    covers the byte after it; a run of backslashes reaches the next lane
//    only through its parity (a lane of 16 backslashes passes the carry on);
//  - the string bytes: the unescaped quotes toggle between outside and
//    inside (the run starts outside every string), the parity of those in
//    the lanes before coming from a ballot;
//  - the output: string j of the run (its 32-bit length, then its decoded
//    bytes) starts at O0 + 4 j + R, R the decoded bytes of the run's strings
//    before it, from one wave scan of each lane's (strings opened, bytes).
// A run whose bytes hold something this does not decode, or does not decode
// the same way as the per-string scan, is left to the per-string path: a
// byte below 0x20 in a string, a bad escape or \u sequence, a backslash
// outside strings, or quotes that do not open a string exactly at each
// string entry and close it before its document ends.  The counting pass
// records which runs were left; the writing pass follows that.
constexpr uint32_t kRingBytes = 2048;  // the writing pass's output, per wave (a step adds at most 1366)

struct alignas(16) RunCountLds {  // per wave
  uint32_t epos[kRunMax];   // string j: its entry's position, from the span's base
  uint32_t eend[kRunMax];   // string j: its document's end, from the span's base
  uint32_t val[kRunMax];    // string j: the run's decoded bytes before its opening quote
  uint32_t slen[kRunMax];   // string j: its decoded bytes
};
struct alignas(16) RunWriteLds {  // per wave
  uint32_t val[kRunMax];    // string j: its buffer bytes, as counted
  uint32_t ring[kRingBytes / 4 + 1];  // the output, then a spare word for bytes that write nothing
};

// Bit b of the result: byte b of the 16 bytes in x equals c (a zero-byte test
// per byte: no borrow crosses a byte).
JSIDX_DEV uint32_t bytes_zero(const uint32_t x[4], uint32_t pat, uint32_t keep) {
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t t = (x[k] ^ pat) & keep;
    const uint32_t z = ~(((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
    uint32_t f = z >> 7;  // bits 0, 8, 16, 24 to 0..3
    f |= f >> 7;
    f |= f >> 14;
    r |= (f & 0xFu) << (4 * k);
  }
  return r;
}
JSIDX_DEV uint32_t bytes_eq(const uint32_t x[4], uint32_t c) { return bytes_zero(x, c * 0x01010101u, ~0u); }
JSIDX_DEV uint32_t bytes_ctl(const uint32_t x[4]) { return bytes_zero(x, 0u, 0xE0E0E0E0u); }  // below 0x20
JSIDX_DEV uint32_t byte_in(const uint32_t x[4], uint32_t i) { return (word_in(x, i / 4) >> (8 * (i & 3u))) & 0xFFu; }

// Four hex digits at p of the buffer (below bhi), or -1.
JSIDX_DEV int32_t hex_at(const uint8_t* buf, uint64_t p, uint64_t bhi) {
  if (p + 4 > bhi) return -1;
  int32_t v = 0;
  for (int k = 0; k < 4; k++) {
    const int32_t h = hex_digit(prim::load1(buf + p + k));
    if (h < 0) return -1;
    v = v * 16 + h;
  }
  return v;
}

// Stores output bytes [from, to) of a run (indices from the 16-byte block
// holding its first byte O0, which is byte d of it; from a multiple of 16):
// whole blocks with 16-byte stores, the bytes of partial blocks one by one.
JSIDX_DEV void ring_store(const uint32_t* ring, uint8_t* str, uint64_t O0, uint32_t d, uint32_t from, uint32_t to) {
  const uint32_t nb = to > from ? (to - from + 15) / 16 : 0u;
  const uint8_t* r8 = reinterpret_cast<const uint8_t*>(ring);
  for (uint32_t m = prim::lane(); m < nb; m += 64u) {
    const uint32_t r0 = from + 16 * m;
    if (r0 >= d && r0 + 16 <= to) {
      prim::st_out4(reinterpret_cast<uint32_t*>(str + O0 + (r0 - d)), prim::ld_lds128(ring + (r0 & (kRingBytes - 1)) / 4));
    } else {
      for (uint32_t b = 0; b < 16u; b++) {
        const uint32_t r = r0 + b;
        if (r >= d && r < to) prim::st_byte(str + O0 + (r - d), prim::lds_ld1(r8 + (r & (kRingBytes - 1))));
      }
    }
  }
}

// A run's bytes are read from the 16-byte aligned address at or below its
// start: the span's base.
JSIDX_DEV int64_t span_base(const uint8_t* buf, uint64_t p0) {
  return (int64_t)p0 - (int64_t)(reinterpret_cast<uintptr_t>(buf + p0) & 15u);
}
// This lane's 16 bytes of step `step` of a span (whole 16-byte loads inside
// [blo, bhi), single bytes at the buffer's ends, 0 outside).
JSIDX_DEV uint4 span_load(const uint8_t* buf, int64_t base, uint32_t step, uint64_t blo, uint64_t bhi) {
  const int64_t pb = base + 1024ll * step + 16ll * prim::lane();
  if (pb >= (int64_t)blo && pb + 16 <= (int64_t)bhi) return prim::load16(buf + pb);
  uint32_t x[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int b = 0; b < 16; b++)
    if (pb + b >= (int64_t)blo && pb + b < (int64_t)bhi) x[b / 4] |= prim::load1(buf + pb + b) << (8 * (b % 4));
  return uint4{x[0], x[1], x[2], x[3]};
}
JSIDX_DEV uint32_t span_steps(int64_t base, uint64_t p1) { return (uint32_t)(((int64_t)p1 - base + 1023) / 1024); }

// The run's strings, in its bytes from p0 (its first entry) to p1 (the entry
// after the run, or the buffer's end), nstr of them; [blo, bhi) is the
// readable buffer; s0 and s1 this lane's bytes of the first two steps,
// loaded by the caller (later steps are loaded one step ahead).  Counting
// (!WRITE): T.epos and T.eend hold the string entries; fills T.slen.
// Writing: T.val holds each string's buffer bytes; stores the run's output
// from buffer offset O0 on.  Returns whether the run was left to the
// per-string path (the same for the whole wave; when counting only).
template <bool WRITE, class Tables>
JSIDX_DEV bool fast_run(Tables& T, const uint8_t* buf, uint64_t p0, uint64_t p1, uint64_t blo, uint64_t bhi,
                        uint32_t nstr, uint8_t* str, uint64_t O0, uint4 s0, uint4 s1) {
  const uint32_t lane = prim::lane();
  const uint64_t below = (1ull << lane) - 1u;
  const int64_t base = span_base(buf, p0);
  const uint32_t nsteps = span_steps(base, p1);
  uint32_t ecarry = 0, pcarry = 0, ocarry = 0, J = 0, R = 0;  // carries into the next step
  bool bad = false;
  uint32_t d = 0, flushed = 0;
  if constexpr (WRITE) d = (uint32_t)(reinterpret_cast<uintptr_t>(str + O0) & 15u);
  uint4 cur = s0, nxt = s1;
  for (uint32_t step = 0; step < nsteps && !bad; step++) {
    const int64_t pb = base + 1024ll * step + 16ll * lane;
    const uint32_t x[4] = {cur.x, cur.y, cur.z, cur.w};
    cur = nxt;
    if (step + 2 < nsteps) nxt = span_load(buf, base, step + 2, blo, bhi);
    // the run's bytes: [p0, p1)
    const int64_t vlo = (int64_t)p0 - pb, vhi = (int64_t)p1 - pb;
    uint32_t valid = 0xFFFFu;
    if (vlo > 0) valid = vlo >= 16 ? 0u : (0xFFFFu << vlo) & 0xFFFFu;
    if (vhi < 16) valid &= vhi <= 0 ? 0u : (1u << vhi) - 1u;
    const uint32_t qm = bytes_eq(x, '"') & valid, bm = bytes_eq(x, '\\') & valid;
    // bytes below 0x20 (only where some lane has one: rare in a minified
    // document); a byte below 0x20 sets its top bit in x - 0x20.. and not in x
    bool any_ctl = false;
#pragma unroll
    for (int k = 0; k < 4; k++) any_ctl |= ((x[k] - 0x20202020u) & ~x[k] & 0x80808080u) != 0u;
    const uint32_t cm = prim::ballot(any_ctl) ? bytes_ctl(x) & valid : 0u;
    bool bad_l = false;
    // escapes
    const bool all_bs = bm == 0xFFFFu;
    const uint32_t top = (uint32_t)__builtin_clz(~(bm << 16));  // backslashes ending the lane
    const uint64_t np = prim::ballot(!all_bs), gm = prim::ballot((top & 1u) != 0u);
    const uint64_t npb = np & below;
    const uint32_t ein = npb ? (uint32_t)(gm >> (63 - __builtin_clzll(npb))) & 1u : ecarry;
    ecarry = np ? (uint32_t)(gm >> (63 - __builtin_clzll(np))) & 1u : ecarry;
    uint32_t esc = 0, st = 0, rem = bm;
    if (ein) {
      esc = 1u;
      rem &= ~1u;
    }
    while (rem) {
      const uint32_t i = (uint32_t)__builtin_ctz(rem);
      st |= 1u << i;
      esc |= 2u << i;
      rem &= ~((4u << i) - 1u);
    }
    esc &= 0xFFFFu;
    // \u escapes: the letter's lane reads the four digits (and, after a high
    // surrogate, the low one's escape) from the document; the bytes they
    // cover may run into the next lane, 10 at most.  A first pass finds how
    // far each lane's escapes run over.  A byte covered from the lane before
    // can only be the low half of a pair, among the lane's first 10 bytes,
    // and an escape there runs over nothing, so the second pass, which skips
    // the covered bytes, runs over the same.
    const uint32_t um = prim::ballot(esc != 0u) ? bytes_eq(x, 'u') & valid : 0u;  // only under escapes
    const uint32_t ue = esc & um;
    uint32_t cov = 0, extra = 0, over = 0;
    uint32_t upos[3] = {16u, 16u, 16u}, uval[3] = {0u, 0u, 0u}, un[3] = {0u, 0u, 0u};
    bool ubad = false;
    auto scan_u = [&](uint32_t covered) {
      cov = covered;
      extra = over = 0;
      ubad = false;
      uint32_t r = ue & ~covered;
#pragma unroll
      for (int t = 0; t < 3; t++) {
        upos[t] = 16u;
        if (r) {
          const uint32_t u = (uint32_t)__builtin_ctz(r);
          const uint64_t P = (uint64_t)(pb + u);
          int32_t cp = hex_at(buf, P + 1, bhi);
          uint32_t c = 4;
          if (cp >= 0xD800 && cp <= 0xDBFF) {
            const int32_t lo = P + 7 <= bhi && prim::load1(buf + P + 5) == '\\' && prim::load1(buf + P + 6) == 'u'
                                   ? hex_at(buf, P + 7, bhi) : -1;
            if (lo >= 0xDC00 && lo <= 0xDFFF) {
              cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
              c = 10;
            } else {
              cp = -1;
            }
          } else if (cp >= 0xDC00 && cp <= 0xDFFF) {
            cp = -1;
          }
          if (cp < 0) {
            ubad = true;
          } else {
            uint32_t nb = 0;
            uval[t] = utf8_of((uint32_t)cp, &nb);
            un[t] = nb;
            upos[t] = u;
            extra += nb - 1;
            cov |= (((1u << c) - 1u) << (u + 1)) & 0xFFFFu;
            if (u + c > 15u && u + c - 15u > over) over = u + c - 15u;
          }
          r &= ~cov & ~((2u << u) - 1u);
        }
      }
      if (r) ubad = true;
    };
    if (ue) scan_u(0u);
    const uint32_t up = prim::shfl_up(over, 1);
    const uint32_t cin = lane == 0 ? ocarry : up;
    ocarry = prim::readlane(over, 63);
    if (cin) {
      const uint32_t first = over;
      scan_u((1u << cin) - 1u);
      if (over != first) ubad = true;
    }
    if (ubad) bad_l = true;
    // string bytes: the unescaped quotes toggle
    const uint32_t uq = qm & ~esc & ~cov;
    const uint64_t pm = prim::ballot((__builtin_popcount(uq) & 1) != 0);
    const uint32_t pin = ((uint32_t)__builtin_popcountll(pm & below) & 1u) ^ pcarry;
    pcarry ^= (uint32_t)__builtin_popcountll(pm) & 1u;
    uint32_t px = uq;
    px ^= px << 1;
    px ^= px << 2;
    px ^= px << 4;
    px ^= px << 8;
    const uint32_t inside = (px ^ (pin ? 0xFFFFu : 0u)) & 0xFFFFu;
    const uint32_t opn = uq & inside, cls = uq & ~inside, content = inside & ~uq;
    if ((cm & content) || ((st | esc) & ~content)) bad_l = true;
    for (uint32_t el = esc & ~um; el; el &= el - 1u)
      if (escape_char(byte_in(x, (uint32_t)__builtin_ctz(el))) == 0x100u) bad_l = true;
    // the lane's decoded bytes and opened strings, and those before it
    const uint32_t outm = content & ~st & ~cov;
    const uint32_t v = ((uint32_t)__builtin_popcount(opn) << 16) | ((uint32_t)__builtin_popcount(outm) + extra);
    const uint32_t incl = prim::incl_scan(v);
    const uint32_t Jl = J + ((incl - v) >> 16), Rl = R + ((incl - v) & 0xFFFFu);
    const uint32_t tot = prim::readlane(incl, 63);
    J += tot >> 16;
    R += tot & 0xFFFFu;
    auto r_at = [&](uint32_t i) {  // the run's decoded bytes before byte i of the lane
      uint32_t r = Rl + (uint32_t)__builtin_popcount(outm & ((1u << i) - 1u));
#pragma unroll
      for (int t = 0; t < 3; t++) r += upos[t] < i ? un[t] - 1u : 0u;
      return r;
    };
    if constexpr (!WRITE) {
      for (uint32_t o = opn; o; o &= o - 1u) {
        const uint32_t i = (uint32_t)__builtin_ctz(o);
        const uint32_t j = Jl + (uint32_t)__builtin_popcount(opn & ((1u << i) - 1u));
        if (j >= nstr || T.epos[j] != (uint32_t)(pb + i - base)) bad_l = true;
        else T.val[j] = r_at(i);
      }
      prim::wave_sync();
      for (uint32_t o = cls; o; o &= o - 1u) {
        const uint32_t i = (uint32_t)__builtin_ctz(o);
        const uint32_t jo = Jl + (uint32_t)__builtin_popcount(opn & ((1u << i) - 1u));  // strings opened before
        if (jo == 0 || jo > nstr || (uint32_t)(pb + i - base) >= T.eend[jo - 1]) bad_l = true;
        else T.slen[jo - 1] = r_at(i) - T.val[jo - 1];
      }
    } else if (upos[0] == 16u) {
      // no \u escape in the lane: every plain byte written (bytes that write
      // nothing go to a spare slot, so that the 16 stores need no branch),
      // then the escaped letters and the length words
      uint8_t* ring = reinterpret_cast<uint8_t*>(T.ring);
      const uint32_t o0 = d + 4 * Jl + Rl, plain = outm & ~esc;
      uint32_t o = o0;  // byte b's place: o0, plus 1 per output byte and 4 per string opened before it
#pragma unroll
      for (int b = 0; b < 16; b++) {
        prim::lds_st1(ring + ((plain >> b) & 1u ? (o & (kRingBytes - 1)) : kRingBytes), (x[b / 4] >> (8 * (b % 4))) & 0xFFu);
        o += ((outm >> b) & 1u) + 4u * ((opn >> b) & 1u);
      }
      for (uint32_t e = outm & esc; e; e &= e - 1u) {
        const uint32_t b = (uint32_t)__builtin_ctz(e), mb = (1u << b) - 1u;
        const uint32_t o = o0 + (uint32_t)__builtin_popcount(outm & mb) + 4u * (uint32_t)__builtin_popcount(opn & mb);
        prim::lds_st1(ring + (o & (kRingBytes - 1)), escape_char(byte_in(x, b)));
      }
      for (uint32_t e = opn; e; e &= e - 1u) {
        const uint32_t b = (uint32_t)__builtin_ctz(e), mb = (1u << b) - 1u;
        const uint32_t k = (uint32_t)__builtin_popcount(opn & mb);
        const uint32_t o = o0 + (uint32_t)__builtin_popcount(outm & mb) + 4u * k;
        const uint32_t len = (Jl + k < nstr ? T.val[Jl + k] : 4u) - 4u;
        for (uint32_t q = 0; q < 4u; q++) prim::lds_st1(ring + ((o + q) & (kRingBytes - 1)), (len >> (8 * q)) & 0xFFu);
      }
    } else {
      uint8_t* ring = reinterpret_cast<uint8_t*>(T.ring);
      uint32_t jj = Jl, rr = Rl;
#pragma unroll
      for (int b = 0; b < 16; b++) {
        const uint32_t bit = 1u << b;
        if (opn & bit) {  // the string's length word
          const uint32_t o = d + 4 * jj + rr, len = (jj < nstr ? T.val[jj] : 4u) - 4u;
          for (uint32_t k = 0; k < 4u; k++) prim::lds_st1(ring + ((o + k) & (kRingBytes - 1)), (len >> (8 * k)) & 0xFFu);
          jj++;
        } else if (outm & bit) {
          const uint32_t ch = (x[b / 4] >> (8 * (b % 4))) & 0xFFu;
          uint32_t val = ch, n = 1;
          if (esc & bit) {
            val = escape_char(ch);
#pragma unroll
            for (int t = 0; t < 3; t++)
              if (upos[t] == (uint32_t)b) {
                val = uval[t];
                n = un[t];
              }
          }
          const uint32_t o = d + 4 * jj + rr;
          for (uint32_t k = 0; k < n; k++) prim::lds_st1(ring + ((o + k) & (kRingBytes - 1)), (val >> (8 * k)) & 0xFFu);
          rr += n;
        }
      }
    }
    if constexpr (WRITE) {
      prim::wave_sync();
      const uint32_t done = (d + 4 * J + R) & ~15u;  // whole blocks written
      ring_store(T.ring, str, O0, d, flushed, done);
      flushed = done > flushed ? done : flushed;
      prim::wave_sync();
    }
    bad = prim::ballot(bad_l) != 0u;
  }
  if constexpr (WRITE) {
    ring_store(T.ring, str, O0, d, flushed, d + 4 * J + R);
    prim::wave_sync();
  }
  return bad || pcarry != 0u || J != nstr;
}

// ---- Literals ---------------------------------------------------------------
JSIDX_DEV bool literal_ok(const TapeArgs& a, const Window& w, uint64_t p, uint32_t first) {
  // true, false, null by their bytes (little-endian words)
  const uint32_t L = first == 'f' ? 5u : 4u;
  if (p + L > a.len) return false;
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

// Eight digits at once (Sec. 3.2.1): the window's bytes p .. p + 7 as one
// little-endian word, if all eight lie in the window and the document.
JSIDX_DEV bool win8(const Window& w, uint64_t p, uint64_t* v) {
  if (w.base == ~0ull || p < w.base || p + 8 > w.len) return false;
  const uint64_t d = p - w.base;
  if (d + 8 > 32) return false;
  const uint32_t k = (uint32_t)(d >> 3), sh = 8u * (uint32_t)(d & 7u);
  const uint64_t lo = pick4(w.q0, w.q1, w.q2, w.q3, k);
  const uint64_t hi = pick4(w.q0, w.q1, w.q2, w.q3, k + 1u);  // 0 past the window
  *v = sh ? (lo >> sh) | (hi << (64u - sh)) : lo;
  return true;
}
// All eight bytes are '0'..'9': each byte's high nibble is 3 and adding 6
// keeps it 3.
JSIDX_DEV bool eight_digits(uint64_t v) {
  return (((v & 0xF0F0F0F0F0F0F0F0ull) | (((v + 0x0606060606060606ull) & 0xF0F0F0F0F0F0F0F0ull) >> 4)) ==
          0x3333333333333333ull);
}
// Their value, first digit most significant: neighbouring digits combined
// into pairs, pairs into fours, fours into eight (three multiply-adds).
JSIDX_DEV uint64_t eight_value(uint64_t v) {
  v -= 0x3030303030303030ull;
  v = (v * 10u + (v >> 8)) & 0x00FF00FF00FF00FFull;
  v = (v * 100u + (v >> 16)) & 0x0000FFFF0000FFFFull;
  return (v * 10000u + (v >> 32)) & 0xFFFFFFFFull;
}

JSIDX_DEV NumText scan_number(const TapeArgs& a, const Window& w, uint64_t p) {
  NumText t{false, false, true, false, 0, 0, 0};
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
      uint64_t v8 = 0;
      if (nd + 8 <= 19 && win8(w, p, &v8) && eight_digits(v8)) {
        t.w = t.w * 100000000ull + eight_value(v8);
        nd += 8;
        t.int_digits += 8;
        p += 8;
        c = win_byte(w, p);
        continue;
      }
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
      uint64_t v8 = 0;
      if (nd > 0 && nd + 8 <= 19 && win8(w, p, &v8) && eight_digits(v8)) {
        t.w = t.w * 100000000ull + eight_value(v8);
        nd += 8;
        q -= 8;
        p += 8;
        c = win_byte(w, p);
        continue;
      }
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
  uint64_t send;   // the next chunk's first buffer byte
  uint32_t qbase[2];  // the workgroup's first slots for its numbers and its literals
  uint32_t gq[kTapeChunk / 64];  // numbers | literals << 16 per group of 64, then their exclusive prefix
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

// The same over one chunk, by 32-bit wave scans and then the four wave
// totals (two barriers).  When some thread's values reach 2^23 (so that the
// sums might not fit 32 bits) the whole workgroup takes group_scan2 instead.
template <typename G>
JSIDX_DEV void chunk_scan2(G& g, uint32_t tid, uint64_t w, uint64_t s, uint64_t* wex, uint64_t* sex,
                           uint64_t* wall, uint64_t* sall) {
  static_assert(kTapeThreads == 256, "four waves");
  constexpr uint64_t kBig = 1ull << 23, kFlag = 1ull << 63;
  const bool big = prim::ballot(w >= kBig || s >= kBig) != 0ull;
  const uint32_t wi = prim::incl_scan((uint32_t)w), si = prim::incl_scan((uint32_t)s), wv = tid / 64u;
  if ((tid & 63u) == 63u) {
    g.w[wv] = (uint64_t)wi | (big ? kFlag : 0ull);
    g.s[wv] = si;
  }
  prim::sync();
  uint32_t wb = 0, sb = 0, wt = 0, st = 0;
  bool any_big = false;
#pragma unroll
  for (uint32_t k = 0; k < 4u; k++) {
    const uint64_t x = g.w[k];
    const uint32_t y = (uint32_t)g.s[k];
    any_big |= (x & kFlag) != 0ull;
    wb += k < wv ? (uint32_t)x : 0u;
    sb += k < wv ? y : 0u;
    wt += (uint32_t)x;
    st += y;
  }
  prim::sync();
  if (any_big) {  // the same for every thread
    group_scan2(g, tid, w, s, wex, sex, wall, sall);
    return;
  }
  *wex = wb + wi - (uint32_t)w;
  *sex = sb + si - (uint32_t)s;
  *wall = wt;
  *sall = st;
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
// The first half of a number-queue slot: for one document the entry's
// position when the write pass has it (and it is below 2^31), else the entry
// with bit 31 set (entries stay below 2^31); for a batch the virtual entry.
constexpr uint32_t kQueueByEntry = 0x80000000u;
template <bool BATCH>
JSIDX_DEV uint32_t queue_key(bool have_pos, uint64_t pos, uint64_t i) {
  if (BATCH) return (uint32_t)i;
  return have_pos && pos < kQueueByEntry ? (uint32_t)pos : (uint32_t)i | kQueueByEntry;
}
template <bool BATCH>
JSIDX_DEV uint64_t queued_pos(const TapeArgs& a, uint32_t x) {
  if (BATCH) return entry_pos<true>(a, x);
  return (x & kQueueByEntry) ? entry_pos<false>(a, x & ~kQueueByEntry) : x;
}
// Slots of the number queue (the workspace's entries).
template <bool BATCH>
JSIDX_DEV uint32_t queue_cap(const TapeArgs& a) { return BATCH ? a.cap : a.n; }
template <bool BATCH>
JSIDX_DEV uint32_t nchunks_of(const TapeArgs& a) { return BATCH ? prim::ld_agent32(a.vn + 1) : a.nchunks; }
// Tape words of an entry with first byte b and batch flags f: its own, plus
// its document's root words if it is the document's first or last entry.
JSIDX_DEV uint32_t entry_words(uint32_t b, uint32_t f) {
  return words_of(b) + (f & kVFirst ? 1u : 0u) + (f & kVLast ? 1u : 0u);
}

// The readable positions of buf: [buf_lo, buf_hi).
template <bool BATCH>
JSIDX_DEV uint64_t buf_lo(const TapeArgs& a) { return BATCH ? prim::load8(a.offsets) : 0u; }
template <bool BATCH>
JSIDX_DEV uint64_t buf_hi(const TapeArgs& a) { return BATCH ? prim::load8(a.offsets + a.ndocs) : a.len; }

// LDS of the counting pass: the workgroup's scan and, per wave, the tables
// of the byte-parallel path or the per-string path's staged bytes.
union alignas(16) CountWaveLds {
  StrLds s;
  RunCountLds r;
};
struct TapeCountLds {
  TapeScanLds sc;
  CountWaveLds w[kTapeThreads / 64];
};

// Each wave takes 512 consecutive entries of a chunk as two runs of
// kTapeSuper groups of 64 (one entry per lane); the loads for all the
// entries of a run (positions, documents, links) are issued together before
// any of them is used, so that a run costs a few memory round trips, not a
// few per group.

// Element q of a per-group array held in registers, by mask arithmetic (a
// runtime index, or a chain of selects the compiler may turn into one, would
// put the array in private memory).
template <typename T>
JSIDX_DEV T pick_group(const T (&v)[kTapeSuper], int q) {
  T r = 0;
#pragma unroll
  for (int j = 0; j < kTapeSuper; j++) r |= v[j] & (T)(0 - (T)(q == j));
  return r;
}

// The first entry of run h of this wave in chunk c.
JSIDX_DEV uint64_t run_first(uint32_t c, int h) {
  return (uint64_t)c * kTapeChunk +
         ((uint64_t)prim::wave_id() * (kTapePer / kTapeSuper) + (uint64_t)h) * (64u * kTapeSuper);
}

// Index of this lane's entry among the run's strings (sm: the strings of
// each group, q: this lane's group).
JSIDX_DEV uint32_t run_index(const uint64_t (&sm)[kTapeSuper], int q) {
  uint32_t k = 0;
#pragma unroll
  for (int j = 0; j < kTapeSuper; j++) k += j < q ? (uint32_t)__builtin_popcountll(sm[j]) : 0u;
  return k + prim::mbcnt(pick_group(sm, q));
}

// The position of the run's first string (whole wave; sm as above, pos the
// lanes' positions per group).
JSIDX_DEV uint64_t run_first_string(const uint64_t (&sm)[kTapeSuper], const uint64_t (&pos)[kTapeSuper]) {
  int q = kTapeSuper - 1;
#pragma unroll
  for (int j = kTapeSuper - 1; j >= 0; j--) q = sm[j] ? j : q;
  return readlane64(pick_group(pos, q), __builtin_ctzll(pick_group(sm, q)));
}

// 1. First bytes and string sizes, their sums per chunk.  A run's strings
//    take the byte-parallel path unless it leaves them to the per-string one
//    (recorded for the writing pass).
template <bool BATCH>
JSIDX_DEV void tape_count(const TapeArgs& a) {
  TapeCountLds& g = prim::lds_object<TapeCountLds>();
  CountWaveLds& W = g.w[prim::wave_id()];
  const uint32_t tid = tape_tid(), lane = prim::lane();
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  const uint64_t blo = buf_lo<BATCH>(a), bhi = buf_hi<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  uint64_t w = 0, s = 0;
  for (int h = 0; h < kTapePer / kTapeSuper; h++) {
    const uint64_t e0 = run_first(c, h);
    if (e0 >= n) break;  // the same for the whole wave
    uint64_t pos[kTapeSuper], len[kTapeSuper], sm[kTapeSuper];
    uint32_t fl[kTapeSuper], by[kTapeSuper], sl[kTapeSuper];
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const uint64_t i = e0 + 64u * q + lane;
      const bool in = i < n;
      fl[q] = BATCH && in ? prim::load1(a.vflag + i) : 0u;
      pos[q] = in ? entry_pos<BATCH>(a, i) : 0u;
      len[q] = !BATCH ? a.len : in ? prim::load8(a.offsets + entry_doc<BATCH>(a, i) + 1) : 0u;
    }
    const uint64_t e1 = e0 + 64u * kTapeSuper;
    const uint64_t p1 = e1 < n ? entry_pos<BATCH>(a, e1) : bhi;
    // the first bytes, and the first two steps of the run's bytes in flight together
    const uint64_t p0 = readlane64(pos[0], 0);
    const int64_t sbase0 = span_base(a.buf, p0);
    const uint32_t nsteps = span_steps(sbase0, p1);
    const uint4 s0 = span_load(a.buf, sbase0, 0, blo, bhi);
    const uint4 s1 = nsteps > 1 ? span_load(a.buf, sbase0, 1, blo, bhi) : uint4{0u, 0u, 0u, 0u};
    uint32_t nstr = 0;
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const bool in = e0 + 64u * q + lane < n;
      by[q] = !in ? 0u : (fl[q] & kVEmpty) ? (uint32_t)':' : pos[q] < len[q] ? prim::load1(a.buf + pos[q]) : 0u;
      sm[q] = prim::ballot(by[q] == '"');
      nstr += (uint32_t)__builtin_popcountll(sm[q]);
      sl[q] = 0;
    }
    bool slow = false;
    if (nstr) {
      // the byte-parallel path, given each string entry's place
      const uint64_t base = (uint64_t)sbase0;
      prim::wave_sync();  // the previous run's reads are done
#pragma unroll
      for (int q = 0; q < kTapeSuper; q++) {
        if (by[q] == '"') {
          const uint32_t k = run_index(sm, q);
          W.r.epos[k] = (uint32_t)(pos[q] - base);
          W.r.eend[k] = len[q] - base < 0xFFFFFFFFull ? (uint32_t)(len[q] - base) : 0xFFFFFFFFu;
        }
      }
      prim::wave_sync();
      slow = fast_run<false>(W.r, a.buf, p0, p1, blo, bhi, nstr, nullptr, 0u, s0, s1);
      prim::wave_sync();
      if (!slow) {
#pragma unroll
        for (int q = 0; q < kTapeSuper; q++)
          if (by[q] == '"') sl[q] = W.r.slen[run_index(sm, q)];
      }
      if (lane == 0) prim::st_byte(a.runbad + e0 / kRunMax, slow ? 1u : 0u);
    }
    if (!slow) {
#pragma unroll
      for (int q = 0; q < kTapeSuper; q++) {
        const uint64_t i = e0 + 64u * q + lane;
        if (i >= n) continue;
        const uint32_t sb = by[q] == '"' ? 4 + sl[q] : 0u;
        prim::st_out(a.sbytes + i, sb);
        prim::st_byte(a.kb + i, by[q]);
        w += entry_words(by[q], fl[q]);
        s += sb;
      }
      continue;
    }
    // the per-string path
    StrSrc src = stage_group(W.s, a.buf, run_first_string(sm, pos), p1, blo, bhi);
    for (int q = 0; q < kTapeSuper; q++) {
      if (e0 + 64u * q >= n) break;  // the same for the whole wave
      const uint64_t i = e0 + 64u * q + lane;
      const bool in = i < n;
      const uint32_t b = pick_group(by, q);
      src.len = pick_group(len, q);
      uint32_t slen = 0;
      (void)wave_strings<false>(src, W.s, in && b == '"', pick_group(pos, q), StrDst{nullptr, 0u, false}, &slen);
      if (!in) continue;
      const uint32_t sb = b == '"' ? 4 + slen : 0u;
      prim::st_out(a.sbytes + i, sb);
      prim::st_byte(a.kb + i, b);
      w += entry_words(b, pick_group(fl, q));
      s += sb;
    }
  }
  uint64_t wex, sex, wall, sall;
  chunk_scan2(g.sc, tid, w, s, &wex, &sex, &wall, &sall);
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
  // each thread's run of chunks, eight loads in flight at a time
  constexpr int kB = 8;
  uint64_t w = 0, s = 0;
  for (uint64_t c = lo; c < hi; c += kB) {
    uint64_t vw[kB], vs[kB];
#pragma unroll
    for (int k = 0; k < kB; k++) {
      vw[k] = c + k < hi ? ld64(a.chunk_sum + 2 * (c + k)) : 0u;
      vs[k] = c + k < hi ? ld64(a.chunk_sum + 2 * (c + k) + 1) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kB; k++) {
      w += vw[k];
      s += vs[k];
    }
  }
  uint64_t wex, sex, wall, sall;
  group_scan2(g, tid, w, s, &wex, &sex, &wall, &sall);
  for (uint64_t c = lo; c < hi; c += kB) {
    uint64_t vw[kB], vs[kB];
#pragma unroll
    for (int k = 0; k < kB; k++) {
      vw[k] = c + k < hi ? ld64(a.chunk_sum + 2 * (c + k)) : 0u;
      vs[k] = c + k < hi ? ld64(a.chunk_sum + 2 * (c + k) + 1) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kB; k++) {
      if (c + k < hi) {
        st64(a.chunk_sum + 2 * (c + k), wex);
        st64(a.chunk_sum + 2 * (c + k) + 1, sex);
      }
      wex += vw[k];
      sex += vs[k];
    }
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

// Stages chunk c (first bytes and string sizes, each thread's run of 8
// entries in wide loads) and turns them into each entry's tape index (T) and
// buffer offset (S) by a scan over the runs.  (For a batch, T is the index of the
// entry's own first word, after its document's opening root word if it is
// the document's first entry; F holds the batch flags.)
template <bool BATCH>
JSIDX_DEV void stage_offsets(const TapeArgs& a, uint32_t n, TapeChunkT<BATCH>& g, uint32_t tid, uint32_t c) {
  const uint64_t c0 = (uint64_t)c * kTapeChunk;
  const uint32_t j0 = tid * (uint32_t)kTapePer;
  const uint64_t e = c0 + j0;
  // the thread's 8 entries in wide loads (past n: ':', no bytes, no flags)
  uint32_t k8[2] = {0x3A3A3A3Au, 0x3A3A3A3Au}, f8[2] = {0u, 0u}, sv[kTapePer];
  if (e + kTapePer <= n) {
    const uint2 kv = prim::ld_pair(reinterpret_cast<const uint2*>(a.kb + e));
    const uint4 s0 = prim::load16(reinterpret_cast<const uint8_t*>(a.sbytes + e));
    const uint4 s1 = prim::load16(reinterpret_cast<const uint8_t*>(a.sbytes + e + 4));
    k8[0] = kv.x;
    k8[1] = kv.y;
    sv[0] = s0.x, sv[1] = s0.y, sv[2] = s0.z, sv[3] = s0.w;
    sv[4] = s1.x, sv[5] = s1.y, sv[6] = s1.z, sv[7] = s1.w;
    if (BATCH) {
      const uint2 fv = prim::ld_pair(reinterpret_cast<const uint2*>(a.vflag + e));
      f8[0] = fv.x;
      f8[1] = fv.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kTapePer; k++) {
      const bool in = e + k < n;
      const uint32_t sh = 8u * (uint32_t)(k & 3), keep = ~(0xFFu << sh);
      if (in) k8[k / 4] = (k8[k / 4] & keep) | (prim::load1(a.kb + e + k) << sh);
      sv[k] = in ? prim::load4(reinterpret_cast<const uint8_t*>(a.sbytes + e + k)) : 0u;
      if (BATCH && in) f8[k / 4] |= prim::load1(a.vflag + e + k) << sh;
    }
  }
  uint32_t kb[kTapePer], fl[kTapePer];
  uint64_t w = 0, s = 0;
#pragma unroll
  for (int k = 0; k < kTapePer; k++) {
    kb[k] = (k8[k / 4] >> (8 * (k & 3))) & 0xFFu;
    fl[k] = (f8[k / 4] >> (8 * (k & 3))) & 0xFFu;
    g.K[j0 + k] = (uint8_t)kb[k];
    if (BATCH) g.F[j0 + k] = (uint8_t)fl[k];
    w += BATCH ? entry_words(kb[k], fl[k]) : words_of(kb[k]);
    s += sv[k];
  }
  uint64_t wex, sex, wall, sall;
  chunk_scan2(g.sc, tid, w, s, &wex, &sex, &wall, &sall);
  uint64_t tw = (BATCH ? 0 : 1) + ld64(a.chunk_sum + 2 * (uint64_t)c) + wex;
  uint64_t ts = ld64(a.chunk_sum + 2 * (uint64_t)c + 1) + sex;
#pragma unroll
  for (int k = 0; k < kTapePer; k++) {
    const uint32_t first = BATCH && (fl[k] & kVFirst) ? 1u : 0u;
    if (BATCH && first && e + k < n) {
      // the document's bases: its opening root word and its first string byte
      const uint32_t d = prim::load4(reinterpret_cast<const uint8_t*>(a.docid + e + k));
      st64(a.dbase + 2 * (uint64_t)d, tw);
      st64(a.dbase + 2 * (uint64_t)d + 1, ts);
    }
    g.T[j0 + k] = (uint32_t)(tw + first);
    g.S[j0 + k] = (uint32_t)ts;  // the buffer offset's low word (see tape_write)
    tw += BATCH ? entry_words(kb[k], fl[k]) : words_of(kb[k]);
    ts += sv[k];
  }
  if (tid == kTapeThreads - 1) g.send = ts;
  prim::sync();
}

// 3. The tape index of each bracket (the only entries whose index another
//    chunk looks up: their partners'), stored coalesced.  (A batch also
//    writes each document's bases here, which needs the string sizes.)
template <bool BATCH>
JSIDX_DEVFN void tape_offsets(const TapeArgs& a) {
  TapeChunkT<BATCH>& g = prim::lds_object<TapeChunkT<BATCH>>();
  const uint32_t tid = tape_tid();
  if (!batch_go<BATCH>(a)) return;
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
    const uint64_t c0 = (uint64_t)c * kTapeChunk;
    if (!BATCH) {
      // one document: each thread's 8 entries from one 8-byte load of their
      // first bytes (past n they read as ':', which has no word)
      const uint64_t e = c0 + (uint64_t)tid * kTapePer;
      uint32_t lo = 0x3A3A3A3Au, hi = 0x3A3A3A3Au;
      if (e + kTapePer <= n) {
        const uint2 v = prim::ld_pair(reinterpret_cast<const uint2*>(a.kb + e));
        lo = v.x;
        hi = v.y;
      } else {
        for (int k = 0; k < kTapePer; k++) {
          if (e + k >= n) break;
          const uint32_t sh = 8u * (uint32_t)(k & 3), b = prim::load1(a.kb + e + k);
          if (k < 4) lo = (lo & ~(0xFFu << sh)) | (b << sh);
          else hi = (hi & ~(0xFFu << sh)) | (b << sh);
        }
      }
      uint32_t w = 0;
#pragma unroll
      for (int k = 0; k < kTapePer; k++) w += words_of(((k < 4 ? lo : hi) >> (8 * (k & 3))) & 0xFFu);
      uint64_t wex, sex, wall, sall;
      chunk_scan2(g.sc, tid, w, 0u, &wex, &sex, &wall, &sall);
      uint32_t t = (uint32_t)(1u + ld64(a.chunk_sum + 2 * (uint64_t)c) + wex);
#pragma unroll
      for (int k = 0; k < kTapePer; k++) {
        const uint32_t b = ((k < 4 ? lo : hi) >> (8 * (k & 3))) & 0xFFu;
        if (is_bracket(b)) prim::st_out(a.toff + e + k, t);
        t += words_of(b);
      }
      continue;
    }
    stage_offsets<BATCH>(a, n, g, tid, c);
    for (uint32_t j = tid; j < (uint32_t)kTapeChunk; j += kTapeThreads) {
      if (c0 + j >= n) break;
      if (is_bracket(g.K[j])) prim::st_out(a.toff + c0 + j, g.T[j]);
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

// LDS of the writing pass: the chunk and, per wave, the byte-parallel
// path's sizes and output or the per-string path's staged bytes.
union alignas(16) WriteWaveLds {
  StrLds s;
  RunWriteLds r;
};
template <bool BATCH>
struct TapeWriteLds {
  TapeChunkT<BATCH> ch;
  WriteWaveLds w[kTapeThreads / 64];
};

// The strings of a group of 64 entries (whole wave; `has`: this lane's entry
// is a string at pos, in a document ending at len, whose output, the length
// word and the bytes, takes sz buffer bytes from offset so, as counted), read
// through src.  Returns the lane's error flags.
JSIDX_DEV uint32_t write_strings(const TapeArgs& a, StrLds& L, StrSrc src, bool has, uint64_t pos, uint64_t len,
                                 uint64_t so, uint64_t sz) {
  const int f = __builtin_ctzll(prim::ballot(has));  // the group's first string
  src.len = len;
  // the group's output is contiguous from the first string's on; the strings
  // that fit in kStrOut bytes with it (a prefix of them) are staged
  const uint64_t A = readlane64(so, f);
  const uint32_t d = (uint32_t)(reinterpret_cast<uintptr_t>(a.str + A) & 15u);
  const uint64_t rel = so - A + d;
  const bool staged = has && rel + sz <= kStrOut;
  const StrDst o{a.str + so + 4, (uint32_t)(staged ? rel + 4 : 0u), staged};
  prim::wave_sync();  // the previous group's output is stored
  uint32_t cnt = 0;
  const uint32_t err = wave_strings<true>(src, L, has, pos, o, &cnt);
  if (has) {
    for (uint32_t j = 0; j < 4u; j++) {  // the length word
      const uint32_t v = (cnt >> (8 * j)) & 0xFFu;
      if (staged) prim::lds_st1(reinterpret_cast<uint8_t*>(L.out) + rel + j, v);
      else prim::st_byte(a.str + so + j, v);
    }
  }
  const uint64_t sm = prim::ballot(staged);
  if (sm) copy_out(L, a.str, A, readlane64(so + sz, 63 - __builtin_clzll(sm)), d);
  return err;
}

// numbers and literals
JSIDX_DEV bool is_queued(uint32_t b) { return !in_set(b, kNoWordLo | set_lo('"'), kBracketHi); }

// 4. Brackets, strings and the strings' words; numbers and literals queued
//    with their tape indices (one atomic per workgroup).  In a batch, links
//    and string offsets are relative to the entry's document's tape and
//    strings.
template <bool BATCH>
JSIDX_DEV void tape_write(const TapeArgs& a) {
  TapeWriteLds<BATCH>& G = prim::lds_object<TapeWriteLds<BATCH>>();
  TapeChunkT<BATCH>& g = G.ch;
  WriteWaveLds& W = G.w[prim::wave_id()];
  const uint32_t tid = tape_tid(), lane = prim::lane();
  if (!batch_go<BATCH>(a)) return;
  const uint32_t n = n_of<BATCH>(a), nchunks = nchunks_of<BATCH>(a);
  const uint64_t blo = buf_lo<BATCH>(a), bhi = buf_hi<BATCH>(a);
  for (uint32_t c = prim::block(); c < nchunks; c += prim::grid()) {
  stage_offsets<BATCH>(a, n, g, tid, c);
  const uint64_t c0 = (uint64_t)c * kTapeChunk;
  // the workgroup's slots in the queue, in entry order (so that the number
  // pass's windows and tape words of a wave lie close together), numbers
  // from the queue's front and literals from its back (so that a wave of the
  // number pass takes one kind, not both paths): counts per group of 64
  // entries, their prefix over the chunk
  const uint32_t gw = (uint32_t)(run_first(c, 0) - c0) / 64u;  // this wave's first group
  for (int k = 0; k < kTapePer; k++) {
    const uint32_t b = g.K[64u * (gw + k) + lane];  // entries past n were staged as ':'
    const uint32_t nl = (uint32_t)__builtin_popcountll(prim::ballot(is_lit_start(b)));
    const uint32_t nn = (uint32_t)__builtin_popcountll(prim::ballot(is_queued(b) && !is_lit_start(b)));
    if (lane == 0) g.gq[gw + k] = nn | (nl << 16);
  }
  prim::sync();
  if (tid < 64u) {
    const uint32_t v = tid < (uint32_t)(kTapeChunk / 64) ? g.gq[tid] : 0u;
    const uint32_t incl = prim::incl_scan(v);  // each half stays below 2^16: 2048 entries a chunk
    const uint32_t all = prim::readlane(incl, 63);
    if (tid == 0) {
      g.qbase[0] = (all & 0xFFFFu) ? prim::add_agent32(a.qcount + 1, all & 0xFFFFu) : 0u;
      g.qbase[1] = (all >> 16) ? prim::add_agent32(a.qcount + 2, all >> 16) : 0u;
    }
    prim::wave_sync();
    if (tid < (uint32_t)(kTapeChunk / 64)) g.gq[tid] = incl - v;
  }
  prim::sync();
  // a chunk's buffer bytes stay below 2^32 (its strings lie in the input,
  // fewer than 2^32 - 2^16 bytes), so an offset is the chunk base plus its
  // low word's distance from the base's
  const uint64_t sbase = ld64(a.chunk_sum + 2 * (uint64_t)c + 1);
  for (int h = 0; h < kTapePer / kTapeSuper; h++) {
    const uint64_t e0 = run_first(c, h);
    if (e0 >= n) break;  // the same for the whole wave
    const uint32_t j0 = (uint32_t)(e0 - c0);
    // the run's loads: documents, positions and links, then the documents'
    // bases and (batches) links, then the partners' tape indices
    uint32_t dq[kTapeSuper], mq[kTapeSuper], v0q[kTapeSuper], limq[kTapeSuper];
    uint64_t pos[kTapeSuper], len[kTapeSuper], w0q[kTapeSuper], s0q[kTapeSuper], obq[kTapeSuper];
    bool any_str = false;
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) any_str |= e0 + 64u * q + lane < n && g.K[j0 + 64u * q + lane] == '"';
    const bool run_str = prim::ballot(any_str) != 0u;
    // a run with strings loads its positions anyway: its numbers' positions
    // then go into the number queue too
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const uint64_t i = e0 + 64u * q + lane;
      const uint32_t b = g.K[j0 + 64u * q + lane];
      const bool in = i < n, br = in && is_bracket(b), st = in && b == '"';
      dq[q] = BATCH && (br || st) ? prim::load4(reinterpret_cast<const uint8_t*>(a.docid + i)) : 0u;
      pos[q] = st || (!BATCH && run_str && in && is_queued(b)) ? entry_pos<BATCH>(a, i) : 0u;
      mq[q] = !BATCH && br ? prim::load4(reinterpret_cast<const uint8_t*>(a.match + i)) : kTapeUnlinked;
    }
    const uint64_t e1 = e0 + 64u * kTapeSuper;
    const uint64_t p1 = !run_str ? 0u : e1 < n ? entry_pos<BATCH>(a, e1) : bhi;
    // the byte-parallel path's first two steps, in flight with the loads below
    const bool fast = run_str && prim::load1(a.runbad + e0 / kRunMax) == 0u;
    const uint64_t rp0 = fast ? entry_pos<BATCH>(a, e0) : 0u;
    const int64_t sbase0 = span_base(a.buf, rp0);
    const uint32_t nsteps = fast ? span_steps(sbase0, p1) : 0u;
    const uint4 s0 = nsteps > 0 ? span_load(a.buf, sbase0, 0, blo, bhi) : uint4{0u, 0u, 0u, 0u};
    const uint4 s1 = nsteps > 1 ? span_load(a.buf, sbase0, 1, blo, bhi) : uint4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const uint64_t i = e0 + 64u * q + lane;
      const uint32_t b = g.K[j0 + 64u * q + lane];
      const bool in = i < n, br = in && is_bracket(b), st = in && b == '"';
      const uint32_t d = dq[q];
      w0q[q] = BATCH && (br || st) ? ld64(a.dbase + 2 * (uint64_t)d) : 0u;
      s0q[q] = BATCH && st ? ld64(a.dbase + 2 * (uint64_t)d + 1) : 0u;
      len[q] = !BATCH ? a.len : st ? prim::load8(a.offsets + d + 1) : 0u;
      v0q[q] = BATCH && br ? prim::load4(reinterpret_cast<const uint8_t*>(a.vstart + d)) : 0u;
      obq[q] = BATCH && br ? prim::load8(a.offsets + d) : 0u;
      limq[q] = !BATCH ? n : br ? prim::load4(reinterpret_cast<const uint8_t*>(a.dn + d)) : 0u;
    }
    if (BATCH) {
#pragma unroll
      for (int q = 0; q < kTapeSuper; q++) {
        const uint64_t i = e0 + 64u * q + lane;
        const uint32_t b = g.K[j0 + 64u * q + lane];
        const bool br = i < n && is_bracket(b);
        mq[q] = br ? prim::load4(reinterpret_cast<const uint8_t*>(a.match + obq[q] + (i - v0q[q]))) : kTapeUnlinked;
      }
    }
    // the partners' tape indices: from this chunk's staged ones when the
    // partner is in the chunk, else as the offsets pass stored them
    uint32_t tkq[kTapeSuper];
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const bool linked = mq[q] != kTapeUnlinked && mq[q] < limq[q];
      const uint64_t pe = (uint64_t)v0q[q] + mq[q], pj = pe - c0;
      tkq[q] = !linked ? 0u : pj < (uint64_t)kTapeChunk ? g.T[pj] : prim::load4(reinterpret_cast<const uint8_t*>(a.toff + pe));
    }
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const uint32_t j = j0 + 64u * q + lane;
      const uint64_t i = c0 + j;
      const uint32_t b = g.K[j];
      if (i >= n) continue;
      if (is_bracket(b)) {
        uint64_t link = 0;
        if (mq[q] != kTapeUnlinked && mq[q] < limq[q]) {
          const uint64_t tk = tkq[q] - w0q[q];
          link = (b == '{' || b == '[') ? tk + 1 : tk;
        }
        st64(a.tape + g.T[j], ((uint64_t)b << 56) | link);
      }
    }
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const uint32_t j = j0 + 64u * q + lane;
      const uint32_t b = g.K[j];
      const bool in = c0 + j < n, lit = in && is_lit_start(b), num = in && is_queued(b) && !lit;
      const uint64_t mn = prim::ballot(num), ml = prim::ballot(lit);
      const uint32_t gp = g.gq[j / 64u];
      const uint32_t x = queue_key<BATCH>(run_str, pos[q], c0 + j);
      if (num) prim::st_pair(a.nqueue + g.qbase[0] + (gp & 0xFFFFu) + prim::mbcnt(mn), x, g.T[j]);
      if (lit) prim::st_pair(a.nqueue + queue_cap<BATCH>(a) - 1u - (g.qbase[1] + (gp >> 16) + prim::mbcnt(ml)), x, g.T[j]);
    }
    if (!run_str) continue;
    // the strings' words; each string's buffer offset and bytes
    uint64_t sm[kTapeSuper], so[kTapeSuper];
    uint32_t nstr = 0;
#pragma unroll
    for (int q = 0; q < kTapeSuper; q++) {
      const uint32_t j = j0 + 64u * q + lane;
      const bool str = c0 + j < n && g.K[j] == '"';
      so[q] = sbase + (uint32_t)(g.S[j] - (uint32_t)sbase);
      if (str) st64(a.tape + g.T[j], ((uint64_t)'"' << 56) | (so[q] - s0q[q]));
      sm[q] = prim::ballot(str);
      nstr += (uint32_t)__builtin_popcountll(sm[q]);
    }
    if (fast) {
      // the byte-parallel path: the run's output is contiguous from its first entry's offset on
      prim::wave_sync();  // the previous run's reads are done
#pragma unroll
      for (int q = 0; q < kTapeSuper; q++) {
        const uint32_t j = j0 + 64u * q + lane;
        if (c0 + j < n && g.K[j] == '"') {
          const uint64_t so1 = j + 1 < (uint32_t)kTapeChunk ? sbase + (uint32_t)(g.S[j + 1] - (uint32_t)sbase) : g.send;
          W.r.val[run_index(sm, q)] = (uint32_t)(so1 - so[q]);
        }
      }
      prim::wave_sync();
      (void)fast_run<true>(W.r, a.buf, rp0, p1, blo, bhi, nstr, a.str, readlane64(so[0], 0), s0, s1);
      continue;
    }
    // the per-string path, group by group, from the run's staged bytes
    const StrSrc src = stage_group(W.s, a.buf, run_first_string(sm, pos), p1, blo, bhi);
    for (int q = 0; q < kTapeSuper; q++) {
      const uint32_t j = j0 + 64u * q + lane;
      const uint64_t i = c0 + j;
      const bool str = i < n && g.K[j] == '"';
      if (prim::ballot(str) == 0u) continue;  // the same for the whole wave
      const uint64_t sq = pick_group(so, q);
      const uint64_t so1 = j + 1 < (uint32_t)kTapeChunk ? sbase + (uint32_t)(g.S[j + 1] - (uint32_t)sbase) : g.send;
      const uint32_t err = write_strings(a, W.s, src, str, pick_group(pos, q), pick_group(len, q), sq, so1 - sq);
      or_flags<BATCH>(a, err, pick_group(dq, q));
    }
  }
  prim::sync();
  }
}

// Grid-stride bounds of a queue for this thread.
JSIDX_DEV uint32_t queue_len(const TapeArgs& a, int q) { return prim::ld_agent32(a.qcount + q); }

JSIDX_DEV NumText scan_number(const TapeArgs& a, uint64_t p) { return scan_number(a, window_at(a.buf, a.len, p), p); }

// The window of an atom at p: loaded anywhere below hi (for a batch, the
// batch's end, so that the loads need not wait for the document's bounds),
// read only inside the entry's document.
JSIDX_DEV Window atom_window(const TapeArgs& a, uint64_t hi, uint64_t p) {
  Window w = window_at(a.buf, hi, p);
  w.len = a.len;
  return w;
}

// 5. Numbers (both words; undecided doubles queued for tape_exact) and
//    literals.  (a: arguments whose bound is the entry's document; hi the
//    end of the readable bytes; pos its first byte.)
JSIDX_DEV uint32_t number_entry(const TapeArgs& a, uint64_t hi, uint64_t pos, uint64_t t, bool* undecided) {
  uint64_t* out = a.tape + t;
  *undecided = false;
  const Window w = atom_window(a, hi, pos);
  const uint32_t b = win_byte(w, pos);
  if (is_lit_start(b)) {  // a literal: its tag, and whether it is spelled out
    st64(out, (uint64_t)b << 56);
    return literal_ok(a, w, pos, b) ? 0u : kErrLiteral;
  }
  const NumText nt = scan_number(a, w, pos);
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
  const uint32_t qn = queue_len(a, 1), ql = queue_len(a, 2);  // numbers, then literals from the back
  const uint64_t bhi = buf_hi<BATCH>(a);
  const uint32_t stride = prim::grid() * (uint32_t)kTapeThreads;
  const uint32_t rounds = (qn + ql + stride - 1) / stride;
  for (uint32_t r = 0; r < rounds; r++) {
    const uint32_t q = r * stride + prim::block() * (uint32_t)kTapeThreads + tape_tid();
    bool undecided = false;
    uint32_t slot = 0, d = 0, err = 0;
    if (q < qn + ql) {
      slot = q < qn ? q : queue_cap<BATCH>(a) - 1u - (q - qn);
      const uint2 e = prim::ld_pair(a.nqueue + slot);
      d = entry_doc<BATCH>(a, e.x);
      const uint64_t pos = queued_pos<BATCH>(a, e.x);
      err = number_entry(entry_args<BATCH>(a, d), bhi, pos, e.y, &undecided);
    }
    const uint32_t xs = wave_append(a, 0, undecided);
    if (undecided) prim::st_out(a.queue + xs, slot);
    or_flags<BATCH>(a, err, d);
  }
}

// 6. The queued numbers, one thread each, by exact arithmetic.
struct ExactScratch {
  Big D, V, S;
};

template <bool BATCH>
JSIDX_DEV void exact_entry(const TapeArgs& a, uint32_t slot, ExactScratch& x) {
  const uint2 e = prim::ld_pair(a.nqueue + slot);
  const uint32_t d = entry_doc<BATCH>(a, e.x);
  const TapeArgs la = entry_args<BATCH>(a, d);
  const uint64_t pos = queued_pos<BATCH>(a, e.x);
  const uint64_t t = e.y;
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
    // four steps of 64 entries at a time, their loads in flight together
    constexpr uint32_t kU = 4;
    for (uint32_t j0 = 0; j0 < cnt; j0 += kU * 64u) {
      uint32_t pj[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) {
        const uint32_t j = j0 + u * 64u + lane;
        pj[u] = nd && j < cnt ? prim::load4(reinterpret_cast<const uint8_t*>(a.idx + base + j)) : 0u;
      }
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) {
        const uint32_t j = j0 + u * 64u + lane;
        if (j >= cnt) continue;
        uint32_t f = nd ? 0u : kVEmpty;
        if (j == 0) f |= kVFirst;
        if (j + 1 == cnt) f |= kVLast;
        st64(a.vpos + v0 + j, base + pj[u]);
        prim::st_byte(a.vflag + v0 + j, f);
        prim::st_out(a.docid + v0 + j, d);
      }
    }
  }
}

}  // namespace jsidx
