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

JSIDX_DEV uint32_t ge_mask(uint32_t a) { return a >= 32u ? 0u : (~0u << a); }
JSIDX_DEV uint32_t lt_mask(uint32_t a) { return a >= 32u ? ~0u : ((1u << a) - 1u); }

// ---- Bit planes --------------------------------------------------------------
// p[b] bit i = bit b of byte i of the segment (w and p must not alias).  With the segment's bytes as
// planes, every byte class below is a few three-input logic operations on
// whole 32-bit masks (v_bitop3_b32), with no per-byte packing step.
//   1. byte transpose (v_perm_b32): u[k] byte j = segment byte 8j + k;
//   2. three swap stages exchange bit s of the register index with bit s of
//      the bit-in-byte index, so register b ends up holding bit b of byte
//      8j + k at position 8j + k.
JSIDX_DEV void bit_planes(const uint32_t w[8], uint32_t p[8]) {
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const uint32_t A = w[h], B = w[h + 2], C = w[h + 4], D = w[h + 6];
    const uint32_t X = perm(B, A, 0x05010400u), Y = perm(B, A, 0x07030602u);
    const uint32_t Z = perm(D, C, 0x05010400u), W = perm(D, C, 0x07030602u);
    p[4 * h + 0] = perm(Z, X, 0x05040100u);
    p[4 * h + 1] = perm(Z, X, 0x07060302u);
    p[4 * h + 2] = perm(W, Y, 0x05040100u);
    p[4 * h + 3] = perm(W, Y, 0x07060302u);
  }
#pragma unroll
  for (int s = 0; s < 3; s++) {
    const int sh = 1 << s;
    const uint32_t m = s == 0 ? 0x55555555u : (s == 1 ? 0x33333333u : 0x0F0F0F0Fu);
#pragma unroll
    for (int r = 0; r < 8; r++) {
      if (r & sh) continue;
      const uint32_t a = p[r], c = p[r + sh];
      p[r] = bfi(m, a, c << sh);
      p[r + sh] = bfi(m, a >> sh, c);
    }
  }
}

// ---- Byte classes (Sec. 3.1.2) -------------------------------------------
// The paper splits each byte into its two nibbles and combines per-nibble
// lookups; on bit planes the same nibble tests are logic on planes 4..7 (high
// nibble) and 0..3 (low nibble).
struct ClassMasks {
  uint32_t C, W, Q, B;  // structural , : [ ] { } | white space | quote | backslash
};

JSIDX_DEV ClassMasks classify_planes(const uint32_t p[8]) {
  const uint32_t n76 = ~(p[7] | p[6]);
  const uint32_t H0 = n76 & ~(p[5] | p[4]);   // 0x0_
  const uint32_t H2 = n76 & p[5] & ~p[4];     // 0x2_
  const uint32_t H3 = n76 & p[5] & p[4];      // 0x3_
  const uint32_t H57 = ~p[7] & p[6] & p[4];   // 0x5_ or 0x7_
  const uint32_t n32 = ~(p[3] | p[2]);
  const uint32_t L0 = n32 & ~(p[1] | p[0]);
  const uint32_t L2 = n32 & p[1] & ~p[0];
  const uint32_t LC = p[3] & p[2] & ~(p[1] | p[0]);
  const uint32_t LA = p[3] & ~p[2] & p[1] & ~p[0];
  const uint32_t LBD = p[3] & p[0] & (p[2] ^ p[1]);                               // B, D
  const uint32_t L9AD = p[3] & ((~p[2] & (p[1] ^ p[0])) | (p[2] & ~p[1] & p[0]));  // 9, A, D
  ClassMasks m;
  m.Q = H2 & L2;                                        // 22
  m.B = H57 & ~p[5] & LC;                               // 5C
  m.C = (H2 & LC) | (H3 & LA) | (H57 & LBD);            // 2C 3A 5B 5D 7B 7D
  m.W = (H2 & L0) | (H0 & L9AD);                        // 20 09 0A 0D
  return m;
}

// The same classes by one comparison per class character and byte, ORed: the
// non-vectorized classification the paper measures against (App. B).  Kept
// out of line (the segment's words passed by value, in registers) so that its
// temporaries do not raise the register pressure of the whole row loop.
struct SegWords {
  uint32_t w[8];
};

__attribute__((noinline)) JSIDX_DEV ClassMasks classify_bytes(SegWords sw) {
  ClassMasks m{0u, 0u, 0u, 0u};
#pragma unroll
  for (int j = 0; j < 32; j++) {
    const uint32_t b = (sw.w[j >> 2] >> (8 * (j & 3))) & 0xFFu;
    const uint32_t c = (b == 0x2Cu) | (b == 0x3Au) | (b == 0x5Bu) | (b == 0x5Du) | (b == 0x7Bu) | (b == 0x7Du);
    const uint32_t s = (b == 0x20u) | (b == 0x09u) | (b == 0x0Au) | (b == 0x0Du);
    m.C |= c << j;
    m.W |= s << j;
    m.Q |= (uint32_t)(b == 0x22u) << j;
    m.B |= (uint32_t)(b == 0x5Cu) << j;
  }
  return m;
}

// (x << 1) with bit 0 taken from bit 31 of x in the previous lane; lane 0
// takes *cin (0/1), which becomes bit 31 of lane 63's x for the next row.
JSIDX_DEV uint32_t shift_in1(uint32_t x, uint32_t* cin) {
  const uint64_t m = prim::ballot((int32_t)x < 0);
  const uint64_t sh = (m << 1) | (uint64_t)*cin;
  *cin = (uint32_t)(m >> 63);
  return (x << 1) | (prim::lane_bit(sh) ? 1u : 0u);
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

// The same by toggling every bit from each set bit upward, one step per set
// bit (the variant without the ladder).
JSIDX_DEV uint32_t prefix_xor_loop(uint32_t m) {
  uint32_t r = 0;
  while (m) {
    r ^= ~0u << (uint32_t)__builtin_ctz(m);
    m &= m - 1u;
  }
  return r;
}

// ---- UTF-8 (Sec. 3.1.5, table of well-formed sequences) --------------------
// On bit planes: a byte is a continuation (10xxxxxx) exactly where the
// sequence rules require one.  lead = 11xxxxxx needs one continuation after
// it, 111xxxxx a second, 1111xxxx a third; C0, C1 and F5..FF never occur, and
// the byte after E0 / ED / F0 / F4 is restricted to A0..BF / 80..9F / 90..BF
// / 80..8F.  D marks document starts (nothing before them counts), E the last
// byte of a document (a sequence still open there is truncated).  Bits are
// set where an error is detected, inside the document it belongs to.
// Carry state between rows: bit 31 of the shifted masks in the lane before.
struct U8Carry {
  uint32_t l4, x, pa, m1, m2, m3;
};

JSIDX_DEV U8Carry u8_carry_zero() { return U8Carry{0u, 0u, 0u, 0u, 0u, 0u}; }

// Carry state after the last 4 bytes before a segment (byte 3 is the last;
// bytes not in the document must be 0).
JSIDX_DEV U8Carry u8_carry_from_word(uint32_t h) {
  const uint32_t b1 = (h >> 8) & 0xFFu, b2 = (h >> 16) & 0xFFu, b3 = h >> 24;
  U8Carry c;
  c.l4 = b3 >= 0xF0u;
  c.x = (b3 >= 0xE0u) | (b2 >= 0xF0u);
  c.pa = (b3 >= 0xC0u) | (b2 >= 0xE0u) | (b1 >= 0xF0u);
  c.m1 = (b3 == 0xE0u) | (b3 == 0xF0u);
  c.m2 = (b3 == 0xEDu) | (b3 == 0xF4u);
  c.m3 = (b3 == 0xF0u) | (b3 == 0xF4u);
  return c;
}

JSIDX_DEV bool u8_carry_pending(const U8Carry& c) { return (c.l4 | c.x | c.pa) != 0u; }

JSIDX_DEV uint32_t utf8_errors(const uint32_t p[8], uint32_t D, uint32_t E, U8Carry* c) {
  const uint32_t cont = p[7] & ~p[6];
  const uint32_t lead = p[7] & p[6];
  const uint32_t L3 = lead & p[5];
  const uint32_t L4 = L3 & p[4];
  const uint32_t A1 = shift_in1(L4, &c->l4) & ~D;        // a 4-byte lead one back
  const uint32_t A2 = shift_in1(L3 | A1, &c->x) & ~D;    // 3+ lead one back or 4-byte two back
  const uint32_t PA = lead | A2;                         // the next byte must continue
  const uint32_t need = shift_in1(PA, &c->pa) & ~D;
  uint32_t err = (cont ^ need) | (PA & E);
  err |= lead & ~(p[5] | p[4] | p[3] | p[2] | p[1]);     // C0, C1
  err |= L4 & (p[3] | (p[2] & (p[1] | p[0])));           // F5..FF
  const uint32_t lowz = ~(p[3] | p[2] | p[1] | p[0]);
  const uint32_t x3 = L3 & ~p[4];                        // E0..EF
  const uint32_t E0 = x3 & lowz;
  const uint32_t ED = x3 & p[3] & p[2] & ~p[1] & p[0];
  const uint32_t F0 = L4 & lowz;
  const uint32_t F4 = L4 & ~p[3] & p[2] & ~p[1] & ~p[0];
  const uint32_t m1 = shift_in1(E0 | F0, &c->m1) & ~D;   // low second bytes are errors
  const uint32_t m2 = shift_in1(ED | F4, &c->m2) & ~D;   // high second bytes are errors
  const uint32_t m3 = shift_in1(F0 | F4, &c->m3) & ~D;   // 4-byte lead: the bound is 0x90
  const uint32_t hi4 = m3 & p[4];
  err |= (m1 & ~p[5] & ~hi4) | (m2 & (p[5] | hi4));
  return err;
}

}  // namespace jsidx
