"""An independent transcription of the paper's 64-bit block formulas.

Used only to pin the byte-at-a-time oracle: the tests run both on the same
inputs and compare.  Nothing here is shared with the oracle or the HIP path.

Sec. 3.1 of Langdale & Lemire processes the input in blocks and gives, for one
block, the bit formulas of Fig. 3 (odd-length backslash runs, using the even /
odd position constants and an add that carries along each run), Fig. 4 (quoted
range as the prefix XOR of the unescaped quotes) and Fig. 5 (structural and
pseudo-structural characters).  Classification uses the two nibble tables of
Sec. 3.1.2.  The paper says state crosses blocks but elides how; this module
supplies the carries in the most direct way:

* escape: if the previous block leaves the next byte escaped, bit 0 of this
  block is escaped (a backslash there is consumed, so it starts no run).  The
  carry out is read from the Fig. 3 formulas evaluated one bit wider than the
  block, with a non-backslash in the extra bit: the OD bit there says whether
  the byte after the block is escaped.
* in-string: the prefix XOR of the previous block's last bit is XORed into
  every bit of this block's R.
* predecessor: the P = S|W bit of the previous block's last byte is shifted
  into bit 0 by the P<<1 step; the byte before the document counts as white
  space.

The functions take masks as Python ints or numpy uint64 arrays, so the same
code serves the single printed example (64-bit blocks, Python ints) and the
vectorised brute force (narrow blocks, numpy).
"""
from __future__ import annotations

import numpy as np

# Sec. 3.1.2: low-nibble and high-nibble lookup tables, as printed.
NIBBLE_LO = [16, 0, 0, 0, 0, 0, 0, 0, 0, 8, 10, 4, 1, 12, 0, 0]
NIBBLE_HI = [8, 0, 17, 2, 0, 4, 0, 4, 0, 0, 0, 0, 0, 0, 0, 0]


def nibble_class(b: int) -> int:
    """Table-driven class value of one byte: lo[b & 15] AND hi[b >> 4]."""
    return NIBBLE_LO[b & 15] & NIBBLE_HI[b >> 4]


_CLASS = np.array([nibble_class(b) for b in range(256)], dtype=np.uint8)


def even_bits(width: int) -> int:
    """The paper's E constant (bits at even offsets), `width` bits wide."""
    return sum(1 << i for i in range(0, width, 2))


def fig3_odd_ends(B, width, one):
    """Fig. 3 at the given width: OD marks the byte after each odd-length run.

    `one` is the all-ones value of the mask type restricted to `width` bits.
    """
    E = even_bits(width) if isinstance(one, int) else np.uint64(even_bits(width))
    O = one & ~E
    S = B & ~(B << 1) & one
    ES = S & E
    EC = (B + ES) & one
    ECE = EC & ~B
    OD1 = ECE & ~E
    OS = S & O
    OC = (B + OS) & one
    OCE = OC & ~B
    OD2 = OCE & E
    return (OD1 | OD2) & one


def prefix_xor(m, width, one):
    """Inclusive prefix XOR by the shift/XOR ladder (App. B)."""
    s = 1
    while s < width:
        m = (m ^ (m << s)) & one
        s *= 2
    return m


def _ones(width, like):
    if isinstance(like, int):
        return (1 << width) - 1
    return np.uint64((1 << width) - 1) if width < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)


def _sh(x, k, like):
    return x << (k if isinstance(like, int) else np.uint64(k))


def block_step(C, W, Qraw, B, nbits, carry, like):
    """Apply Figs. 3-5 to one block of `nbits` bytes.

    C, W, Qraw, B: structural / white-space / quote / backslash masks of the
    block (bit i = byte i).  carry = (esc, in_str, pred).  Returns
    (final mask, rows dict, new carry).
    """
    esc_c, str_c, pred_c = carry
    is_int = isinstance(like, int)
    one = _ones(nbits, like)
    one_w = _ones(nbits + 1, like) if (is_int or nbits + 1 <= 64) else None
    u = (lambda v: v) if is_int else np.uint64
    # Fig. 3 evaluated one bit wider: bit `nbits` is a non-backslash.
    Bp = B & ~esc_c  # an escaped backslash at byte 0 starts no run
    OD_w = fig3_odd_ends(Bp, nbits + 1, one_w)
    OD = (OD_w | esc_c) & one
    esc_out = (OD_w >> u(nbits)) & u(1)
    # Fig. 4.
    Q = Qraw & ~OD
    R = prefix_xor(Q, nbits, one)
    R = R ^ (one * str_c)
    str_out = (R >> u(nbits - 1)) & u(1)
    # Fig. 5.
    S = C & ~R
    S = S | Q
    P = (S | W) & one
    pred_out = (P >> u(nbits - 1)) & u(1)
    P = (_sh(P, 1, like) | pred_c) & one
    P = P & ~W & ~R
    S = S | P
    F = S & ~(Q & ~R) & one
    rows = {"OD": OD, "Q_UNESC": Q, "R": R, "S_OR_Q": C & ~R | Q, "P_MASKED": P, "FINAL": F}
    return F, rows, (esc_out, str_out, pred_out)


def index_strings(X: np.ndarray, width: int):
    """Block-formula index of n equal-length strings at block width `width`.

    X: uint8 array (n, L), L <= 64, width <= 63.  Returns (mask, unclosed,
    trailing_escape) as uint64 arrays: mask bit i = byte i is indexed.
    """
    n, L = X.shape
    cls = _CLASS[X]
    Cb = (cls & 7) != 0
    Wb = (cls & 0x18) != 0
    Qb = X == 0x22
    Bb = X == 0x5C
    zero = np.zeros(n, dtype=np.uint64)
    carry = (zero, zero, np.ones(n, dtype=np.uint64))
    total = np.zeros(n, dtype=np.uint64)
    in_str_final = zero
    for k0 in range(0, L, width):
        nb = min(width, L - k0)
        def pack(M):
            v = np.zeros(n, dtype=np.uint64)
            for j in range(nb):
                v |= M[:, k0 + j].astype(np.uint64) << np.uint64(j)
            return v
        F, rows, carry = block_step(pack(Cb), pack(Wb), pack(Qb), pack(Bb), nb, carry, zero)
        total |= F << np.uint64(k0)
        in_str_final = carry[1]
    return total, in_str_final, carry[0]
