"""Driver for the CPU emulation of the indexing kernel (test infrastructure).

Builds tests/cpu_emu/harness.cpp together with the product kernel body and
runs it through ctypes on host buffers laid out like device memory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "cpu_emu", "harness.cpp")
OUT_DIR = os.path.join(HERE, "cpu_emu", "_build")
LIB = os.path.join(OUT_DIR, "libjsidx_emu.so")
# indexing kernel variants: naive classification, loop prefix XOR, direct flatten
VARIANTS = (1, 2, 4)
_lib = None


def _deps():
    csrc = os.path.join(ROOT, "paper_1902_08318_amd", "csrc")
    files = [SRC, os.path.join(HERE, "cpu_emu", "jsidx_prims.h"), os.path.join(ROOT, "include", "jsidx.h")]
    files += [os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".h")]
    return files


# Builds with other compile-time parameters of the one-document kernel, by
# name (the library's own values are the defaults of jsidx_doc.h).
DOC_BUILDS = {
    "slots2": ["-DJSIDX_DOC_SLOTS=2", "-DJSIDX_DOC_WAVES=4", "-DJSIDX_DOC_BATCH=4"],
    "rows4": ["-DJSIDX_DOC_ROWS=4", "-DJSIDX_DOC_AHEAD=1"],
    "waves4b3": ["-DJSIDX_DOC_WAVES=4", "-DJSIDX_DOC_BATCH=3"],
}


def _lib_path(block_tiles):
    if block_tiles is None:
        return LIB
    return LIB.replace(".so", f"_{block_tiles}.so" if isinstance(block_tiles, str) else f"_b{block_tiles}.so")


def build(block_tiles: int | str | None = None) -> str:
    """Build the emulation library; an int block_tiles overrides the look-back
    block size of both kernels (tests use 1 or 2 so that small inputs span
    many blocks), a string names a build of DOC_BUILDS."""
    os.makedirs(OUT_DIR, exist_ok=True)
    lib = _lib_path(block_tiles)
    if block_tiles is None:
        defs = []
    elif isinstance(block_tiles, str):
        defs = DOC_BUILDS[block_tiles]
    else:
        defs = [f"-DJSIDX_BLOCK_TILES={block_tiles}", f"-DJSIDX_DOC_BLOCK={block_tiles}"]
    # built under a private name and renamed, so that parallel test workers
    # never load a half-written library
    tmp = f"{lib}.{os.getpid()}.tmp"
    subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-shared", "-fPIC", "-pthread", *defs,
         "-I", os.path.join(HERE, "cpu_emu"), "-I", os.path.join(ROOT, "include"),
         "-I", os.path.join(ROOT, "paper_1902_08318_amd", "csrc"), "-o", tmp, SRC],
        check=True)
    os.replace(tmp, lib)
    return lib


_libs = {}


def load(block_tiles: int | None = None):
    global _lib
    if block_tiles is None and _lib is not None:
        return _lib
    if block_tiles in _libs:
        return _libs[block_tiles]
    path = _lib_path(block_tiles)
    if not os.path.exists(path) or any(os.path.getmtime(f) > os.path.getmtime(path) for f in _deps()):
        build(block_tiles)
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.emu_run.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_uint32, vp, ctypes.c_uint64, vp, vp,
                            ctypes.c_int, vp, ctypes.c_uint64, ctypes.c_uint32, vp, vp, ctypes.c_int, ctypes.c_int]
    lib.emu_run.restype = ctypes.c_long
    lib.emu_scopes_run.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_uint32, vp, vp, vp, ctypes.c_int]
    lib.emu_scopes_run.restype = ctypes.c_long
    lib.emu_tape_run.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_uint32, vp, vp, ctypes.c_uint64, vp,
                                 ctypes.c_uint64, vp, vp, vp, vp, ctypes.c_int, vp]
    lib.emu_tape_run.restype = ctypes.c_long
    lib.emu_number.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_int, vp]
    lib.emu_number.restype = ctypes.c_int
    lib.emu_tape_ws_bytes.argtypes = [ctypes.c_uint64]
    lib.emu_tape_ws_bytes.restype = ctypes.c_uint64
    lib.emu_tape_runbad_offset.argtypes = [ctypes.c_uint64]
    lib.emu_tape_runbad_offset.restype = ctypes.c_uint64
    lib.emu_tape_batch_runbad_offset.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.emu_tape_batch_runbad_offset.restype = ctypes.c_uint64
    lib.emu_scopes_ws_bytes.argtypes = [ctypes.c_uint64]
    lib.emu_scopes_ws_bytes.restype = ctypes.c_uint64
    lib.emu_tape_batch_ws_bytes.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.emu_tape_batch_ws_bytes.restype = ctypes.c_uint64
    lib.emu_tape_batch_run.argtypes = [vp, vp, ctypes.c_uint32, vp, vp, vp, vp, ctypes.c_uint64, vp, ctypes.c_uint64,
                                       vp, vp, vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.emu_tape_batch_run.restype = ctypes.c_long
    lib.emu_scopes_batch_ws_bytes.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.emu_scopes_batch_ws_bytes.restype = ctypes.c_uint64
    lib.emu_scopes_batch_run.argtypes = [vp, vp, ctypes.c_uint32, vp, vp, vp, vp, vp, ctypes.c_uint64, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int]
    lib.emu_scopes_batch_run.restype = ctypes.c_long
    lib.emu_ws_bytes.argtypes = [ctypes.c_uint64]
    lib.emu_ws_bytes.restype = ctypes.c_uint64
    lib.emu_tile_bytes.restype = ctypes.c_uint32
    lib.emu_doc_tile_bytes.restype = ctypes.c_uint32
    lib.emu_doc_slots.restype = ctypes.c_uint32
    lib.emu_doc_run.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_uint64, vp, vp, ctypes.c_int, vp, ctypes.c_uint64,
                                vp, vp, ctypes.c_int]
    lib.emu_doc_run.restype = ctypes.c_long
    lib.emu_pick_rows.argtypes = [ctypes.c_int64, ctypes.c_uint64]
    lib.emu_pick_rows.restype = ctypes.c_uint32
    if block_tiles is None:
        _lib = lib
    _libs[block_tiles] = lib
    return lib


def tile_bytes() -> int:
    """Bytes of the largest tile."""
    return int(load().emu_tile_bytes())


def pick_rows(span: int, waves: int) -> int:
    return int(load().emu_pick_rows(span, waves))


class Workspace:
    def __init__(self, cap_tiles: int, block_tiles: int | None = None):
        self.cap = cap_tiles
        self.block_tiles = block_tiles
        self.mem = np.zeros(int(load(block_tiles).emu_ws_bytes(cap_tiles)) // 8 + 1, dtype=np.uint64)


def _aligned(nbytes: int, shift: int) -> tuple[np.ndarray, int]:
    """A zero-filled uint8 buffer whose element `shift` is 64-byte aligned + shift."""
    raw = np.zeros(nbytes + 256, dtype=np.uint8)
    addr = raw.ctypes.data
    off = (-addr) % 64 + shift
    return raw, off


def run(data: bytes, offsets=None, nblocks: int = 2, misalign: int = 0, ws: Workspace | None = None,
        garbage: int = 0xEE, block_tiles: int | None = None, rows: int | None = None, minify: bool = False,
        variant: int = 0):
    """Index `data` (one document if offsets is None, else a batch).

    misalign: the buffer starts this many bytes past a 64-byte boundary.  The
    bytes around the input inside its 16-byte granules are filled with
    `garbage` so that any influence of them shows up.
    block_tiles: look-back block size of the build (None: the library's).
    rows: rows per tile (None: the largest tile; 0: the kernel picks them).
    minify: run the minify pass; out_idx is then a uint8 array of kept bytes.
    variant: the indexing kernel's variant (0 or one of VARIANTS).
    Returns (out_idx, out_n, out_err, violations).
    """
    if ws is not None:
        block_tiles = ws.block_tiles
    lib = load(block_tiles)
    n = len(data)
    raw, off = _aligned(n + 64, misalign + 16)
    raw[:] = garbage
    raw[off:off + n] = np.frombuffer(data, dtype=np.uint8)
    base = raw.ctypes.data + off
    if offsets is None:
        begin, end = 0, n
        offs = None
        ndocs = 1
    else:
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        ndocs = offs.size - 1
        begin, end = int(offs[0]), int(offs[-1])
    glo = (base + begin) & ~15
    ghi = ((base + end + 15) & ~15) if end > begin else glo
    out_cap = max(end, 1)
    out_idx = np.full(out_cap, 0xEE if minify else 0xDEADBEEF, dtype=np.uint8 if minify else np.uint32)
    out_n = np.full(ndocs, 0xDEADBEEF, dtype=np.uint32)
    out_err = np.full(ndocs, 0xDEADBEEF, dtype=np.uint32)
    tb = tile_bytes()
    need = max(1, (end - begin + 15 + tb - 1) // tb)
    if ws is None:
        ws = Workspace(need, block_tiles)
    v = lib.emu_run(ctypes.c_void_p(base), offs.ctypes.data if offs is not None else None, n, ndocs,
                    out_idx.ctypes.data, out_cap, out_n.ctypes.data, out_err.ctypes.data, nblocks,
                    ws.mem.ctypes.data, ws.cap, tile_bytes() // 2048 if rows is None else rows,
                    ctypes.c_void_p(glo), ctypes.c_void_p(ghi), 1 if minify else 0, variant)
    return out_idx, out_n, out_err, int(v)


def scopes(data: bytes, idx: np.ndarray, far_groups: int = 2, garbage_ws: bool = True):
    """Scope links through the emulated scope kernels.  Returns (match, err,
    violations).  The workspace starts full of garbage (the kernels must not
    rely on it being zero)."""
    lib = load()
    n = int(idx.size)
    buf = np.frombuffer(data, dtype=np.uint8) if data else np.zeros(1, dtype=np.uint8)
    ix = np.ascontiguousarray(idx, dtype=np.uint32) if n else np.zeros(1, dtype=np.uint32)
    match = np.full(max(1, n), 0xABABABAB, dtype=np.uint32)
    err = np.full(1, 0xABABABAB, dtype=np.uint32)
    ws = np.full(int(lib.emu_scopes_ws_bytes(n)) // 4 + 64, 0x5A5A5A5A if garbage_ws else 0, dtype=np.uint32)
    v = lib.emu_scopes_run(buf.ctypes.data, len(data), ix.ctypes.data, n, match.ctypes.data, err.ctypes.data,
                           ws.ctypes.data, far_groups)
    return match[:n], int(err[0]), int(v)


def scopes_batch(data: bytes, offsets: np.ndarray, idx: np.ndarray, n: np.ndarray, cap: int | None = None,
                 chunk_groups: int = 2, doc_groups: int = 2, far_groups: int = 2):
    """Batched scope links through the emulated kernels: idx and the result
    in the batch layout (document d at offsets[d]), n the entry counts.
    Returns (match, err per document, violations); outputs and workspace
    start full of garbage."""
    lib = load()
    nd = offsets.size - 1
    total = int(offsets[-1])
    cap = int(n.sum()) if cap is None else cap
    buf = np.frombuffer(data, dtype=np.uint8) if data else np.zeros(1, dtype=np.uint8)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    ix = np.ascontiguousarray(idx, dtype=np.uint32) if total else np.zeros(1, dtype=np.uint32)
    cnt = np.ascontiguousarray(n, dtype=np.uint32)
    match = np.full(max(1, total), 0xABABABAB, dtype=np.uint32)
    err = np.full(nd, 0xABABABAB, dtype=np.uint32)
    ws = np.full(int(lib.emu_scopes_batch_ws_bytes(cap, nd)) // 4 + 64, 0x5A5A5A5A, dtype=np.uint32)
    v = lib.emu_scopes_batch_run(buf.ctypes.data, offs.ctypes.data, nd, ix.ctypes.data, cnt.ctypes.data,
                                 match.ctypes.data, err.ctypes.data, ws.ctypes.data, cap, chunk_groups, doc_groups,
                                 far_groups)
    return match, err, int(v)


def _shifted(nbytes: int, shift: int, fill: int) -> np.ndarray:
    """nbytes bytes (at least 1) starting `shift` bytes past a 64-byte boundary."""
    raw = np.full(max(1, nbytes) + shift + 128, fill, dtype=np.uint8)
    a = (-raw.ctypes.data) % 64
    return raw[a + shift:a + shift + max(1, nbytes)]


def tape(data: bytes, idx: np.ndarray, match: np.ndarray, exact_groups: int = 2, doc_shift: int = 0,
         str_shift: int = 0, paths: list | None = None):
    """The tape through the emulated tape kernels.  Returns (tape words,
    string buffer, flags, violations, numbers taken by the exact conversion);
    the outputs and the workspace start full of garbage.  The document and
    the string buffer start doc_shift and str_shift bytes past a 64-byte
    boundary.  If `paths` is a list, (runs whose strings took the
    byte-parallel path, runs that took the per-string path) is appended."""
    lib = load()
    n = int(idx.size)
    buf = _shifted(len(data), doc_shift, 0)
    if data:
        buf[:] = np.frombuffer(data, dtype=np.uint8)
    ix = np.ascontiguousarray(idx, dtype=np.uint32) if n else np.zeros(1, dtype=np.uint32)
    mt = np.ascontiguousarray(match, dtype=np.uint32) if n else np.zeros(1, dtype=np.uint32)
    tcap = 2 * n + 2
    scap = len(data) + 2 * n + 4
    words = np.full(tcap, 0xA5A5A5A5A5A5A5A5, dtype=np.uint64)
    sbuf = _shifted(scap, str_shift, 0xA5)
    tn = np.full(1, 0xFFFF, dtype=np.uint64)
    sn = np.full(1, 0xFFFF, dtype=np.uint64)
    err = np.full(1, 0xABABABAB, dtype=np.uint32)
    ws = np.full(int(lib.emu_tape_ws_bytes(n)) // 4 + 64, 0x5A5A5A5A, dtype=np.uint32)
    nx = np.zeros(1, dtype=np.uint32)
    v = lib.emu_tape_run(buf.ctypes.data, len(data), ix.ctypes.data, n, mt.ctypes.data, words.ctypes.data, tcap,
                         sbuf.ctypes.data, scap, tn.ctypes.data, sn.ctypes.data, err.ctypes.data, ws.ctypes.data,
                         exact_groups, nx.ctypes.data)
    if paths is not None:
        o = int(lib.emu_tape_runbad_offset(n))
        rb = ws.view(np.uint8)[o:o + n // 256 + 1]  # one byte per run of 256 entries (runs without strings: unset)
        paths.append((int(np.count_nonzero(rb == 0)), int(np.count_nonzero(rb == 1))))
    return words[:int(tn[0])], sbuf[:int(sn[0])].tobytes(), int(err[0]), int(v), int(nx[0])


def tape_batch(data: bytes, offsets: np.ndarray, idx: np.ndarray, n: np.ndarray, match: np.ndarray,
               cap: int | None = None, tape_cap: int | None = None, str_cap: int | None = None,
               chunk_groups: int = 2, doc_groups: int = 2, exact_groups: int = 2, paths: list | None = None):
    """The batched tape through the emulated kernels (index, counts and links
    in the batch layout).  Returns (words, string buffer, out_pos (ndocs x 4),
    flags per document, violations); outputs and workspace start full of
    garbage.  `paths` as for tape()."""
    lib = load()
    nd = offsets.size - 1
    total = int(offsets[-1])
    ent = int(n.sum())
    cap = ent + nd if cap is None else cap
    tcap = 2 * ent + 2 * nd if tape_cap is None else tape_cap
    scap = total + 2 * ent + 4 if str_cap is None else str_cap
    buf = np.frombuffer(data, dtype=np.uint8) if data else np.zeros(1, dtype=np.uint8)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    ix = np.ascontiguousarray(idx, dtype=np.uint32) if total else np.zeros(1, dtype=np.uint32)
    mt = np.ascontiguousarray(match, dtype=np.uint32) if total else np.zeros(1, dtype=np.uint32)
    cnt = np.ascontiguousarray(n, dtype=np.uint32)
    words = np.full(max(1, tcap), 0xA5A5A5A5A5A5A5A5, dtype=np.uint64)
    sbuf = np.full(max(1, scap), 0xA5, dtype=np.uint8)
    pos = np.full(4 * nd, 0xFFFF, dtype=np.uint64)
    err = np.full(nd, 0xABABABAB, dtype=np.uint32)
    ws = np.full(int(lib.emu_tape_batch_ws_bytes(cap, nd)) // 4 + 64, 0x5A5A5A5A, dtype=np.uint32)
    v = lib.emu_tape_batch_run(buf.ctypes.data, offs.ctypes.data, nd, ix.ctypes.data, cnt.ctypes.data,
                               mt.ctypes.data, words.ctypes.data, tcap, sbuf.ctypes.data, scap, pos.ctypes.data,
                               err.ctypes.data, ws.ctypes.data, cap, chunk_groups, doc_groups, exact_groups)
    if paths is not None:
        o = int(lib.emu_tape_batch_runbad_offset(cap, nd))
        rb = ws.view(np.uint8)[o:o + (ent + nd) // 256 + 1]
        paths.append((int(np.count_nonzero(rb == 0)), int(np.count_nonzero(rb == 1))))
    return words, sbuf.tobytes(), pos.reshape(nd, 4), err, int(v)


def number(text: str, exact: bool):
    """(status, magnitude bits) of the device number conversion on one text:
    status 0 ok, 1 infinite, 2 undecided by the fast path, -1 rejected."""
    lib = load()
    raw = text.encode()
    bits = np.zeros(1, dtype=np.uint64)
    r = lib.emu_number(raw, len(raw), 1 if exact else 0, bits.ctypes.data)
    return int(r), int(bits[0])


def doc_tile_bytes() -> int:
    """Bytes of a tile of the one-document kernel."""
    return int(load().emu_doc_tile_bytes())


def run_doc(data: bytes, nwaves: int = 8, misalign: int = 0, ws: Workspace | None = None, garbage: int = 0xEE,
            block_tiles: int | None = None, variant: int = 0):
    """Index one document with the one-document kernel (jsidx_build's).

    misalign: the buffer starts this many bytes past a 64-byte boundary; the
    bytes around the input inside its 16-byte granules hold `garbage`.
    Returns (out_idx, out_n, out_err, violations)."""
    if ws is not None:
        block_tiles = ws.block_tiles
    lib = load(block_tiles)
    n = len(data)
    raw, off = _aligned(n + 64, misalign + 16)
    raw[:] = garbage
    raw[off:off + n] = np.frombuffer(data, dtype=np.uint8)
    base = raw.ctypes.data + off
    glo = base & ~15
    ghi = ((base + n + 15) & ~15) if n else glo
    out_cap = max(n, 1)
    out_idx = np.full(out_cap, 0xDEADBEEF, dtype=np.uint32)
    out_n = np.full(1, 0xDEADBEEF, dtype=np.uint32)
    out_err = np.full(1, 0xDEADBEEF, dtype=np.uint32)
    tb = tile_bytes()
    need = max(1, (n + 15 + tb - 1) // tb)
    if ws is None:
        ws = Workspace(need, block_tiles)
    v = lib.emu_doc_run(ctypes.c_void_p(base), n, out_idx.ctypes.data, out_cap, out_n.ctypes.data,
                        out_err.ctypes.data, nwaves, ws.mem.ctypes.data, ws.cap, ctypes.c_void_p(glo),
                        ctypes.c_void_p(ghi), variant)
    return out_idx, out_n, out_err, int(v)
