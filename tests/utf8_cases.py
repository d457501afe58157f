"""Inputs that walk the table of well-formed UTF-8 sequences (Sec. 3.1.5),
valid and invalid side, for the device tests.  Test data only: byte strings
and their placement, no part of the method's arithmetic (the expected flags
always come from the oracle)."""
from __future__ import annotations

import itertools

import numpy as np

# Second bytes around every range bound of the table (80 8F 90 9F A0 BF),
# plus a byte below the continuation range and a lead byte.
SECONDS = (0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0x41, 0xC2)
# The same 26 bytes as the oracle's four-byte boundary pin.
BOUNDARY_ALPHABET = (0x00, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF,
                     0xE0, 0xE1, 0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xFF,
                     0x41, 0x22)
# Positions (mod 2048 from the start of the launch's first granule) where a
# sequence starts: across a 32-byte segment edge and across a 2 KiB row edge
# (tiles are whole rows, so these are also tile edges).
RESIDUES = (30, 31, 32, 33, 2045, 2046, 2047, 0, 1, 2, 3)


def lead_sequences(seconds=SECONDS):
    """Every lead byte C0..FF with each second byte, padded with 0x80 to the
    length the lead byte announces (2, 3 or 4; 2 for C0, C1 and F5..FF), so
    that validity turns on the lead and second byte alone."""
    out = []
    for lead in range(0xC0, 0x100):
        need = 2 if lead < 0xE0 else (3 if lead < 0xF0 else (4 if lead < 0xF5 else 2))
        for s in seconds:
            out.append(bytes([lead, s]) + b"\x80" * (need - 2))
    return out


def all_strings(length: int):
    """Every byte string of the given length (1..3) as one flat array."""
    grid = np.array(list(itertools.product(range(256), repeat=min(length, 2))), dtype=np.uint8)
    if length <= 2:
        return grid.reshape(-1)
    # 3 bytes: every first byte in front of every two-byte string
    first = np.repeat(np.arange(256, dtype=np.uint8), grid.shape[0])
    rest = np.tile(grid, (256, 1))
    return np.concatenate([first[:, None], rest], axis=1).reshape(-1)


def equal_length_batch(flat: np.ndarray, length: int):
    """(data, offsets) of the documents of `length` bytes packed in flat."""
    n = flat.size // length
    return flat, np.arange(n + 1, dtype=np.uint64) * np.uint64(length)


def boundary_four_byte_batch():
    flat = np.array(list(itertools.product(BOUNDARY_ALPHABET, repeat=4)), dtype=np.uint8).reshape(-1)
    return equal_length_batch(flat, 4)


def placed_batch(seqs, residues=RESIDUES, lead: int = 0, truncate: bool = True, filler: bytes = b"a",
                 period: int = 2048):
    """A batch of documents, one per (sequence, residue): filler bytes, then
    the sequence starting at a global byte position congruent to the residue
    (mod period, counted from byte 0 of the buffer, which the caller places
    `lead` bytes after an aligned start), then ' 1' so that the sequence is
    not at the document's end.  With truncate, each sequence also appears cut
    short at its document's end (every proper prefix of length >= 1).
    Returns (data bytes, offsets uint64)."""
    parts = []
    offs = [0]
    pos = 0
    for s in seqs:
        tails = [s + b" 1"]
        if truncate:
            tails += [s[:k] for k in range(1, len(s))]
        for r in residues:
            for t in tails:
                g = (lead + pos) % period
                pad = (r - g) % period
                doc = filler * pad + t
                parts.append(doc)
                pos += len(doc)
                offs.append(pos)
    return b"".join(parts), np.array(offs, dtype=np.uint64)
