"""CPU oracle for the stage-1 structural index -- TEST INFRASTRUCTURE ONLY.

Wraps the plain byte-at-a-time C definition in ``jsidx_oracle.c`` (stage 1 of
Langdale & Lemire, "Parsing Gigabytes of JSON per Second", Sec. 3.1, and the
minified form of its dataset-size table) with ctypes.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the HIP library never does.

Flag bits (defined here independently of the HIP library's header):
UTF8 = 0x1, UNCLOSED_STRING = 0x2, TRAILING_ESCAPE = 0x4, EMPTY = 0x8; scope
matching: UNBALANCED = 0x10, MISMATCHED = 0x20; structure: SYNTAX = 0x40;
tape (stage 2, Sec. 3.2): NUMBER = 0x100, STRING = 0x200, LITERAL = 0x400.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

ERR_UTF8 = 0x1
ERR_UNCLOSED_STRING = 0x2
ERR_TRAILING_ESCAPE = 0x4
ERR_EMPTY = 0x8

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jsidx_oracle.c")
_LIB = os.path.join(_HERE, "libjsidx_oracle.so")
_lib = None


def build() -> str:
    """Compile the oracle with the host C compiler (plain -O2, no tuning)."""
    subprocess.run(
        ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
         "-o", _LIB, _SRC],
        check=True)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_index.argtypes = [u8p, ctypes.c_uint64, u32p, u32p]
    lib.oracle_index.restype = ctypes.c_uint32
    lib.oracle_index_batch.argtypes = [u8p, u64p, ctypes.c_uint32, u32p, u32p, u32p]
    lib.oracle_index_batch.restype = ctypes.c_int
    lib.oracle_minify.argtypes = [u8p, ctypes.c_uint64, u8p, u32p]
    lib.oracle_minify.restype = ctypes.c_uint32
    lib.oracle_minify_batch.argtypes = [u8p, u64p, ctypes.c_uint32, u8p, u32p, u32p]
    lib.oracle_minify_batch.restype = ctypes.c_int
    lib.oracle_scopes.argtypes = [u8p, u32p, ctypes.c_uint32, u32p, u32p]
    lib.oracle_scopes.restype = ctypes.c_uint32
    lib.oracle_structure.argtypes = [u8p, u32p, ctypes.c_uint32, u32p]
    lib.oracle_structure.restype = ctypes.c_uint32
    lib.oracle_tape.argtypes = [u8p, ctypes.c_uint64, u32p, ctypes.c_uint32, u64p, u64p, u8p, u64p, u32p]
    lib.oracle_tape.restype = ctypes.c_uint32
    lib.oracle_utf8_valid.argtypes = [u8p, ctypes.c_uint64]
    lib.oracle_utf8_valid.restype = ctypes.c_int
    _lib = lib
    return lib


def _u8(buf) -> np.ndarray:
    if isinstance(buf, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(buf), dtype=np.uint8)
    a = np.ascontiguousarray(buf, dtype=np.uint8)
    return a


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def index(buf) -> tuple[np.ndarray, int]:
    """Index one document. Returns (uint32 positions, flags)."""
    a = _u8(buf)
    out = np.empty(max(1, a.size), dtype=np.uint32)
    err = np.zeros(1, dtype=np.uint32)
    n = _load().oracle_index(_ptr(a, ctypes.c_uint8) if a.size else None, a.size,
                             _ptr(out, ctypes.c_uint32), _ptr(err, ctypes.c_uint32))
    return out[:n].copy(), int(err[0])


def index_batch(bufs, offsets) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Index a batch; document d is bufs[offsets[d]:offsets[d+1]].

    Returns (out_idx, out_n, out_err): out_idx has offsets[-1] entries and doc
    d's positions (relative to its start) are out_idx[offsets[d]:offsets[d]+out_n[d]].
    """
    a = _u8(bufs)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nd = off.size - 1
    if nd < 0:
        raise ValueError("offsets must hold ndocs+1 entries")
    if int(off[-1]) > a.size:
        raise ValueError("offsets exceed buffer")
    out = np.zeros(max(1, int(off[-1])), dtype=np.uint32)
    out_n = np.zeros(max(1, nd), dtype=np.uint32)
    out_err = np.zeros(max(1, nd), dtype=np.uint32)
    rc = _load().oracle_index_batch(
        _ptr(a, ctypes.c_uint8) if a.size else None, _ptr(off, ctypes.c_uint64), nd,
        _ptr(out, ctypes.c_uint32), _ptr(out_n, ctypes.c_uint32),
        _ptr(out_err, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("offsets must be nondecreasing")
    return out[: int(off[-1])], out_n[:nd], out_err[:nd]


def minify(buf) -> tuple[bytes, int]:
    """Minify one document: drop the white-space bytes outside strings.
    Returns (kept bytes, flags)."""
    a = _u8(buf)
    out = np.empty(max(1, a.size), dtype=np.uint8)
    err = np.zeros(1, dtype=np.uint32)
    n = _load().oracle_minify(_ptr(a, ctypes.c_uint8) if a.size else None, a.size,
                              _ptr(out, ctypes.c_uint8), _ptr(err, ctypes.c_uint32))
    return out[:n].tobytes(), int(err[0])


def minify_batch(bufs, offsets) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Minify a batch; document d's kept bytes are out[offsets[d]:offsets[d]+out_n[d]].
    Returns (out uint8, out_n, out_err)."""
    a = _u8(bufs)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nd = off.size - 1
    if nd < 0:
        raise ValueError("offsets must hold ndocs+1 entries")
    if int(off[-1]) > a.size:
        raise ValueError("offsets exceed buffer")
    out = np.zeros(max(1, int(off[-1])), dtype=np.uint8)
    out_n = np.zeros(max(1, nd), dtype=np.uint32)
    out_err = np.zeros(max(1, nd), dtype=np.uint32)
    rc = _load().oracle_minify_batch(
        _ptr(a, ctypes.c_uint8) if a.size else None, _ptr(off, ctypes.c_uint64), nd,
        _ptr(out, ctypes.c_uint8), _ptr(out_n, ctypes.c_uint32), _ptr(out_err, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("offsets must be nondecreasing")
    return out[: int(off[-1])], out_n[:nd], out_err[:nd]


ERR_UNBALANCED = 0x10
ERR_MISMATCHED = 0x20


def scopes(buf, idx) -> tuple[np.ndarray, int]:
    """Scope matching over a document's index (positions idx into buf): the
    partner entry of every bracket (0xFFFFFFFF if unlinked or not a bracket)
    and the flags (UNBALANCED, MISMATCHED)."""
    a = _u8(buf)
    ix = np.ascontiguousarray(idx, dtype=np.uint32)
    n = ix.size
    match = np.empty(max(1, n), dtype=np.uint32)
    stack = np.empty(max(1, n), dtype=np.uint32)
    if n and int(ix.max()) >= a.size:
        raise ValueError("positions exceed the document")
    err = _load().oracle_scopes(_ptr(a, ctypes.c_uint8) if a.size else None, _ptr(ix, ctypes.c_uint32), n,
                                _ptr(match, ctypes.c_uint32), _ptr(stack, ctypes.c_uint32))
    return match[:n].copy(), int(err)


ERR_SYNTAX = 0x40


def structure(buf, idx) -> int:
    """0, or ERR_SYNTAX if the index entries' tokens do not form one JSON value
    (token contents are not checked)."""
    a = _u8(buf)
    ix = np.ascontiguousarray(idx, dtype=np.uint32)
    stack = np.empty(max(1, ix.size), dtype=np.uint32)
    if ix.size and int(ix.max()) >= a.size:
        raise ValueError("positions exceed the document")
    return int(_load().oracle_structure(_ptr(a, ctypes.c_uint8) if a.size else None, _ptr(ix, ctypes.c_uint32),
                                        ix.size, _ptr(stack, ctypes.c_uint32)))


ERR_NUMBER = 0x100
ERR_STRING = 0x200
ERR_LITERAL = 0x400


def tape(buf, idx) -> tuple[np.ndarray, bytes, int]:
    """The stage-2 tape of a document (Sec. 3, Fig. 2) from its index: the
    tape words (uint64), the string buffer, and the flags of the atoms and
    strings (NUMBER, STRING, LITERAL).  The tape and buffer are empty unless
    the structure is valid and no flag is set."""
    a = _u8(buf)
    ix = np.ascontiguousarray(idx, dtype=np.uint32)
    n = ix.size
    if n and int(ix.max()) >= a.size:
        raise ValueError("positions exceed the document")
    words = np.zeros(2 * n + 2, dtype=np.uint64)
    sbuf = np.zeros(a.size + 2 * n + 4, dtype=np.uint8)
    stack = np.empty(max(1, n), dtype=np.uint32)
    tn = np.zeros(1, dtype=np.uint64)
    sn = np.zeros(1, dtype=np.uint64)
    flags = _load().oracle_tape(_ptr(a, ctypes.c_uint8) if a.size else None, a.size, _ptr(ix, ctypes.c_uint32), n,
                                _ptr(words, ctypes.c_uint64), _ptr(tn, ctypes.c_uint64), _ptr(sbuf, ctypes.c_uint8),
                                _ptr(sn, ctypes.c_uint64), _ptr(stack, ctypes.c_uint32))
    return words[:int(tn[0])].copy(), sbuf[:int(sn[0])].tobytes(), int(flags)


def utf8_valid(buf) -> bool:
    """True iff buf is a concatenation of the well-formed UTF-8 sequences of
    the paper's table of code points (Sec. 3.1.5)."""
    a = _u8(buf)
    return bool(_load().oracle_utf8_valid(_ptr(a, ctypes.c_uint8) if a.size else None,
                                          a.size))
