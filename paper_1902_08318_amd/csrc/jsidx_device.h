// Device building blocks of the gfx950 stage-1 indexer: byte classification,
// mask compaction, odd-backslash-run detection, prefix XOR and UTF-8 checks.
//
// A lane owns a 32-byte segment of the input and keeps one 32-bit mask per
// byte class (bit j = byte j of the segment).  All byte-level work is SWAR on
// the eight little-endian 32-bit words of the segment.
#pragma once
#include <stdint.h>

#include <jsidx_prims.h>  // resolved through the include path

namespace jsidx {

JSIDX_DEV uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return prim::perm(hi, lo, sel);
}

JSIDX_DEV uint32_t bfi(uint32_t m, uint32_t a, uint32_t b) {
  return (m & a) | (~m & b);
}

// 0xFF in every byte of v whose top bit is set, 0x00 elsewhere.  v_perm_b32
// selectors 8..11 replicate the sign bit of bytes 1, 3, 5, 7 of its 64-bit
// source; feeding (v << 8, v) exposes the sign of all four bytes of v.
JSIDX_DEV uint32_t signmask(uint32_t v) {
  return perm(v << 8, v, 0x090B080Au);
}

// 0xFF in byte k iff bit k of the low nibble n is set (selector 12 -> 0x00,
// selector 13 -> 0xFF).
JSIDX_DEV uint32_t nibble_bytemask(uint32_t n) {
  uint32_t spread = (n & 1u) | ((n & 2u) << 7) | ((n & 4u) << 14) | ((n & 8u) << 21);
  return perm(0u, 0u, 0x0C0C0C0Cu + spread);
}

JSIDX_DEV uint32_t ge_mask(uint32_t a) { return a >= 32u ? 0u : (~0u << a); }
JSIDX_DEV uint32_t lt_mask(uint32_t a) { return a >= 32u ? ~0u : ((1u << a) - 1u); }

// ---- Byte classes (Sec. 3.1.2) -------------------------------------------
// The class byte of each input byte is looked up from its two nibbles and the
// two results are ANDed, as in the paper's table-driven classification; here
// the tables live in v_perm_b32 operands.  Bits of the class byte:
//   0 quote 0x22 | 1 white space 09 0A 0D | 2 white space 20
//   3 comma 2C | 4 colon 3A | 5 brackets/braces 5B 5D 7B 7D | 6 backslash 5C
// High-nibble table (nibbles 0..7; bytes >= 0x80 are cleared separately):
//   [0]=02 [1]=00 [2]=0D [3]=10 [4]=00 [5]=60 [6]=00 [7]=20
// Low-nibble table (nibbles 0..15):
//   [0]=04 [2]=01 [9]=02 [A]=12 [B]=20 [C]=48 [D]=22, others 00.
// A 16-entry lookup is done with two v_perm_b32 whose halves are selected by
// XORing the nibble with 2 and then with 8: out-of-range selectors yield 0xFF
// (neutral under AND) except selector 12 (0x00), which the XOR with 2 sends to
// nibbles 6 and 14, both of class 0.  Entries at odd table positions carry a
// spare 0x80 bit so that selectors 8..11 also yield 0xFF; bit 7 of the class
// byte is never used.
constexpr uint32_t kHiLo = 0x100D0002u, kHiHi = 0x20006000u;
constexpr uint32_t kT1Lo = 0x80048001u, kT1Hi = 0x80008000u;
constexpr uint32_t kT2Lo = 0x8200A012u, kT2Hi = 0xA2488000u;

struct ClassWord {
  uint32_t cls;   // class byte per input byte
  uint32_t hidx;  // high nibble & 7 per byte (shared with UTF-8 lookups)
  uint32_t sgn;   // 0xFF per byte >= 0x80
};

JSIDX_DEV ClassWord classify_word(uint32_t x) {
  ClassWord c;
  c.hidx = (x >> 4) & 0x07070707u;
  uint32_t rhi = perm(kHiHi, kHiLo, c.hidx);
  uint32_t n1 = (x ^ 0x02020202u) & 0x0F0F0F0Fu;
  uint32_t r1 = perm(kT1Hi, kT1Lo, n1);
  uint32_t r2 = perm(kT2Hi, kT2Lo, n1 ^ 0x08080808u);
  c.sgn = signmask(x);
  c.cls = bfi(c.sgn, 0u, r1 & r2 & rhi);
  return c;
}

// Gather one flag per byte of eight words into a 32-bit mask (bit 4k+j =
// byte j of word k).  Every byte of f[k] holds 0 or (1 << SH); v_dot4_u32_u8
// with weights {1,2,4,8} / {16,32,64,128} packs two words into one byte.
template <int SH>
JSIDX_DEV uint32_t compact8(const uint32_t f[8]) {
  uint32_t b0 = prim::udot4(f[1], 0x80402010u, prim::udot4(f[0], 0x08040201u, 0u));
  uint32_t b1 = prim::udot4(f[3], 0x80402010u, prim::udot4(f[2], 0x08040201u, 0u));
  uint32_t b2 = prim::udot4(f[5], 0x80402010u, prim::udot4(f[4], 0x08040201u, 0u));
  uint32_t b3 = prim::udot4(f[7], 0x80402010u, prim::udot4(f[6], 0x08040201u, 0u));
  uint32_t lo16 = b0 | (b1 << 8);
  uint32_t hi16 = b2 | (b3 << 8);
  return (lo16 >> SH) | (hi16 << (16 - SH));
}

struct ClassMasks {
  uint32_t C, W, Q, B;  // structural, white space, quote, backslash
  uint32_t hi;          // OR of the bytes' top bits (non-ASCII present)
};

JSIDX_DEV ClassMasks classify_segment(const uint32_t w[8], uint32_t hidx[8], uint32_t sgn[8]) {
  uint32_t fq[8], fw[8], fc[8], fb[8];
  uint32_t any = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) {
    ClassWord c = classify_word(w[k]);
    hidx[k] = c.hidx;
    sgn[k] = c.sgn;
    any |= w[k];
    fq[k] = c.cls & 0x01010101u;
    fw[k] = ((c.cls & 0x06060606u) + 0x06060606u) & 0x08080808u;
    fc[k] = ((c.cls & 0x38383838u) + 0x38383838u) & 0x40404040u;
    fb[k] = c.cls & 0x40404040u;
  }
  ClassMasks m;
  m.Q = compact8<0>(fq);
  m.W = compact8<3>(fw);
  m.C = compact8<6>(fc);
  m.B = compact8<6>(fb);
  m.hi = any & 0x80808080u;
  return m;
}

// ---- Odd-length backslash runs (Sec. 3.1.1, Fig. 3) -----------------------
// The paper's even/odd-start construction: runs starting at an even offset
// end an odd-length run when the add carries out to an odd offset, and vice
// versa.  Returns the bytes that immediately follow an odd-length run.
// Carries out of bit 31 are dropped; the caller tracks them.
JSIDX_DEV uint32_t odd_run_ends(uint32_t B) {
  const uint32_t E = 0x55555555u, O = 0xAAAAAAAAu;
  uint32_t S = B & ~(B << 1);
  uint32_t OD1 = ((B + (S & E)) & ~B) & ~E;
  uint32_t OD2 = ((B + (S & O)) & ~B) & E;
  return OD1 | OD2;
}

// Escaped bytes of a 32-byte segment.  D marks document starts (the escape
// state resets there); e_in says whether byte 0 is escaped by the preceding
// bytes of the same document.  *after: bit i set iff byte i+1 would be escaped
// (byte i ends an odd-length run), judged within the piece holding byte i;
// bit 31 is the escape carried into the next segment.
JSIDX_DEV uint32_t escaped_bytes(uint32_t B, uint32_t D, uint32_t e_in, uint32_t* after) {
  uint32_t OD = 0, A = 0;
  uint32_t e = (D & 1u) ? 0u : e_in;
  uint32_t a = 0;
  uint32_t rest = D & ~1u;
  uint32_t last_bp = 0;
  while (true) {
    uint32_t b = rest ? (uint32_t)__builtin_ctz(rest) : 32u;
    uint32_t segm = ge_mask(a) & lt_mask(b);
    uint32_t Bp = B & segm & ~(e << a);  // an escaped backslash starts no run
    uint32_t ends = odd_run_ends(Bp);      // carries land one past each run
    OD |= (ends | (e << a)) & segm;
    A |= (ends >> 1) & segm;
    last_bp = Bp;
    if (b == 32u) break;
    rest &= rest - 1u;
    a = b;
    e = 0;
  }
  uint32_t nb = ~last_bp;
  uint32_t run = nb ? (uint32_t)__builtin_clz(nb) : 32u;  // trailing backslash run
  A |= (run & 1u) << 31;
  *after = A;
  return OD;
}

// Inclusive prefix XOR by the shift/XOR ladder (App. B).
JSIDX_DEV uint32_t prefix_xor(uint32_t m) {
  m ^= m << 1;
  m ^= m << 2;
  m ^= m << 4;
  m ^= m << 8;
  m ^= m << 16;
  return m;
}

// ---- UTF-8 (Sec. 3.1.5, table of well-formed sequences) --------------------
// Each byte is checked against the byte before it with three nibble lookups
// whose AND is non-zero exactly for ill-formed (previous, current) pairs; a
// separate test requires continuation bytes 2 and 3 positions after a 3- and
// 4-byte lead.  Error-class bits (tables derived from the well-formed ranges):
//   01 lead not followed by a continuation   02 continuation after ASCII
//   04 E0 followed by 80..9F                 08 ED followed by A0..BF
//   10 C0/C1 lead                            20 F4 + 90..BF, or F5..FF lead
//   40 F0 + 80..8F, or F5..FF + 80..8F       80 continuation after continuation
// Bit 80 is XORed with the "must be continuation" test, so a third or fourth
// byte passes only where a 3- or 4-byte lead requires it.
// Previous-byte high nibble 8..F (0..7 -> 02):
constexpr uint32_t kU1Hi = 0x610D0111u, kU1Lo = 0x80808080u;
// Current-byte high nibble 8..F (0..7 -> 11):
constexpr uint32_t kU3Hi = 0x11111111u, kU3Lo = 0xBABAB6D6u;
// Previous-byte low nibble 0..7 and 8..F:
constexpr uint32_t kU2aHi = 0xE3E3E3A3u, kU2aLo = 0x838393D7u;
constexpr uint32_t kU2bHi = 0xE3E3EBE3u, kU2bLo = 0xE3E3E3E3u;

struct Utf8Word {
  uint32_t t1, t2, t3, gE, gF;
};

JSIDX_DEV Utf8Word utf8_lookup(uint32_t w, uint32_t hidx, uint32_t sgn) {
  Utf8Word u;
  u.t1 = bfi(sgn, perm(kU1Hi, kU1Lo, hidx), 0x02020202u);
  u.t3 = bfi(sgn, perm(kU3Hi, kU3Lo, hidx), 0x11111111u);
  uint32_t lidx = w & 0x07070707u;
  uint32_t m3 = signmask(w << 4);
  u.t2 = bfi(m3, perm(kU2bHi, kU2bLo, lidx), perm(kU2aHi, kU2aLo, lidx));
  u.gE = w & (w << 1) & (w << 2);  // top bit: byte >= 0xE0
  u.gF = u.gE & (w << 3);          // top bit: byte >= 0xF0
  return u;
}

JSIDX_DEV Utf8Word utf8_lookup_raw(uint32_t w) {
  return utf8_lookup(w, (w >> 4) & 0x07070707u, signmask(w));
}

// Error bits of word `cur` given the word before it.
JSIDX_DEV uint32_t utf8_pair_errors(const Utf8Word& prev, const Utf8Word& cur) {
  uint32_t t1p = prim::alignbyte(cur.t1, prev.t1, 3);
  uint32_t t2p = prim::alignbyte(cur.t2, prev.t2, 3);
  uint32_t special = t1p & t2p & cur.t3;
  uint32_t must = (prim::alignbyte(cur.gE, prev.gE, 2) |
                   prim::alignbyte(cur.gF, prev.gF, 1)) & 0x80808080u;
  return special ^ must;
}

}  // namespace jsidx
