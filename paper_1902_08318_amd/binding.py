"""ctypes binding of libjsidx.so (argument marshalling only).

Every entry point mirrors a function of include/jsidx.h.  Tensors must be
device (HIP) tensors; PyTorch provides the memory and the stream.  There is no
fallback: if the library is not built, importing the functions that need it
raises.
"""
from __future__ import annotations

import ctypes
import os

ERR_UTF8 = 0x1
ERR_UNCLOSED_STRING = 0x2
ERR_TRAILING_ESCAPE = 0x4
ERR_EMPTY = 0x8
ERR_UNBALANCED = 0x10
ERR_MISMATCHED = 0x20
ERR_SYNTAX = 0x40
ERR_NUMBER = 0x100
ERR_STRING = 0x200
ERR_LITERAL = 0x400
ERR_OFFSETS = 0x40000000
ERR_CAPACITY = 0x80000000

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libjsidx.so")
_lib = None

# Every symbol include/jsidx.h declares, with its ctypes signature.
_VP = ctypes.c_void_p
SIGNATURES = {
    "jsidx_build": ([_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_build_batch": ([_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_build_noalloc": ([_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_minify": ([_VP, ctypes.c_uint64, _VP, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_minify_batch": ([_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_scopes": ([_VP, ctypes.c_uint64, _VP, ctypes.c_uint32, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_scopes_batch": ([_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_tape_batch": ([_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, _VP, ctypes.c_uint64, _VP, ctypes.c_uint64, _VP,
                          _VP, _VP], ctypes.c_int),
    "jsidx_tape_reserve": ([ctypes.c_uint64, ctypes.c_uint32, _VP], ctypes.c_int),
    "jsidx_scopes_reserve": ([ctypes.c_uint64, ctypes.c_uint32, _VP], ctypes.c_int),
    "jsidx_reserve": ([ctypes.c_uint64, ctypes.c_uint32, _VP], ctypes.c_int),
    "jsidx_workspace_bytes": ([ctypes.c_uint64, ctypes.c_uint32], ctypes.c_size_t),
    "jsidx_release": ([_VP], ctypes.c_int),
    "jsidx_stream_diag": ([_VP, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "jsidx_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "jsidx_set_tile_rows": ([_VP, ctypes.c_uint32], ctypes.c_int),
    "jsidx_set_variant": ([ctypes.c_uint32], ctypes.c_int),
    "jsidx_tape": ([_VP, ctypes.c_uint64, _VP, ctypes.c_uint32, _VP, _VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "jsidx_tile_rows": ([ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
}


class JsidxError(RuntimeError):
    pass


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libjsidx.so (raises if it has not been built).

    PyTorch is imported first: its wheel carries its own HIP runtime
    (SONAME libamdhip64.so.7, loaded under the file name libamdhip64.so).  Once
    that runtime is in the process, the loader resolves this library's
    dependency on libamdhip64.so.7 to it by SONAME, so device pointers and
    streams from PyTorch are used by the same runtime instance.  Loading this
    library first would bring in a second runtime from /opt/rocm.
    """
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see above)
        if not os.path.exists(_LIB_PATH):
            raise JsidxError(f"{_LIB_PATH} is missing: build it with paper_1902_08318_amd/build.py")
        l = ctypes.CDLL(_LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def _check(rc: int):
    if rc != 0:
        raise JsidxError(f"jsidx error {rc}: {lib().jsidx_status_string(rc).decode()}")


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def build(buf, out_idx, out_n, out_err, stream=None, length=None):
    """jsidx_build on device tensors (buf: uint8; outputs: int32/uint32)."""
    n = buf.numel() if length is None else int(length)
    _check(lib().jsidx_build(_ptr(buf), n, _ptr(out_idx), _ptr(out_n), _ptr(out_err), _stream(stream)))


def build_noalloc(buf, out_idx, out_n, out_err, stream=None, length=None):
    """jsidx_build_noalloc on device tensors (same arguments as build)."""
    n = buf.numel() if length is None else int(length)
    _check(lib().jsidx_build_noalloc(_ptr(buf), n, _ptr(out_idx), _ptr(out_n), _ptr(out_err), _stream(stream)))


NOALLOC_MAX_LEN = 268435440


def build_batch(bufs, offsets, out_idx, out_n, out_err, stream=None):
    """jsidx_build_batch on device tensors (offsets: int64, ndocs+1 entries)."""
    nd = offsets.numel() - 1
    _check(lib().jsidx_build_batch(_ptr(bufs), _ptr(offsets), nd, _ptr(out_idx), _ptr(out_n),
                                   _ptr(out_err), _stream(stream)))


def minify(buf, out, out_n, out_err, stream=None, length=None):
    """jsidx_minify on device tensors (buf, out: uint8; out_n, out_err: int32/uint32)."""
    n = buf.numel() if length is None else int(length)
    _check(lib().jsidx_minify(_ptr(buf), n, _ptr(out), _ptr(out_n), _ptr(out_err), _stream(stream)))


def minify_batch(bufs, offsets, out, out_n, out_err, stream=None):
    """jsidx_minify_batch on device tensors (offsets: int64, ndocs+1 entries; out: uint8)."""
    nd = offsets.numel() - 1
    _check(lib().jsidx_minify_batch(_ptr(bufs), _ptr(offsets), nd, _ptr(out), _ptr(out_n), _ptr(out_err),
                                    _stream(stream)))


def scopes(buf, idx, out_match, out_err, stream=None, n=None, length=None):
    """jsidx_scopes on device tensors: buf (uint8, the document), idx (the
    first n index entries), out_match (n uint32/int32), out_err (1)."""
    n = idx.numel() if n is None else int(n)
    ln = buf.numel() if length is None else int(length)
    _check(lib().jsidx_scopes(_ptr(buf), ln, _ptr(idx), n, _ptr(out_match), _ptr(out_err), _stream(stream)))


def scopes_batch(bufs, offsets, idx, n, out_match, out_err, stream=None, ndocs=None):
    """jsidx_scopes_batch on device tensors: bufs (uint8), offsets (ndocs+1
    int64), idx and out_match in the batch layout, n and out_err (ndocs)."""
    nd = offsets.numel() - 1 if ndocs is None else int(ndocs)
    _check(lib().jsidx_scopes_batch(_ptr(bufs), _ptr(offsets), nd, _ptr(idx), _ptr(n), _ptr(out_match),
                                    _ptr(out_err), _stream(stream)))


def tape_batch(bufs, offsets, idx, n, match, out_tape, out_str, out_pos, out_err, stream=None, ndocs=None):
    """jsidx_tape_batch on device tensors: out_tape (int64/uint64 words) and
    out_str (uint8) give their capacities by their sizes; out_pos holds
    4 * ndocs int64."""
    nd = offsets.numel() - 1 if ndocs is None else int(ndocs)
    _check(lib().jsidx_tape_batch(_ptr(bufs), _ptr(offsets), nd, _ptr(idx), _ptr(n), _ptr(match), _ptr(out_tape),
                                  out_tape.numel(), _ptr(out_str), out_str.numel(), _ptr(out_pos), _ptr(out_err),
                                  _stream(stream)))


def tape_reserve(max_entries: int, max_ndocs: int = 0, stream=None):
    """jsidx_tape_reserve."""
    _check(lib().jsidx_tape_reserve(int(max_entries), int(max_ndocs), _stream(stream)))


def scopes_reserve(max_entries: int, max_ndocs: int = 0, stream=None):
    """jsidx_scopes_reserve."""
    _check(lib().jsidx_scopes_reserve(int(max_entries), int(max_ndocs), _stream(stream)))


def reserve(max_total_len: int, stream=None, max_ndocs: int = 0):
    """jsidx_reserve: the stream's workspace for up to max_total_len bytes in
    up to max_ndocs documents."""
    _check(lib().jsidx_reserve(int(max_total_len), int(max_ndocs), _stream(stream)))


def workspace_bytes(total_len: int, ndocs: int = 0) -> int:
    """jsidx_workspace_bytes."""
    return int(lib().jsidx_workspace_bytes(int(total_len), int(ndocs)))


def release(stream=None):
    _check(lib().jsidx_release(_stream(stream)))


def diag(stream=None) -> int:
    v = ctypes.c_uint32(0)
    _check(lib().jsidx_stream_diag(_stream(stream), ctypes.byref(v)))
    return int(v.value)


def set_tile_rows(rows_by_log2) -> None:
    """jsidx_set_tile_rows: rows per tile by floor(log2(span)) (0 = built-in);
    an empty sequence restores the built-in choice."""
    t = bytes(int(r) for r in rows_by_log2)
    buf = ctypes.create_string_buffer(t, max(1, len(t)))
    _check(lib().jsidx_set_tile_rows(ctypes.cast(buf, ctypes.c_void_p), len(t)))


def tape(buf, idx, match, out_tape, out_tape_n, out_str, out_str_n, out_err, stream=None, n=None, length=None):
    """jsidx_tape on device tensors: buf (uint8 document), idx and match (the
    first n entries and their links), out_tape (>= 2n + 2 int64), out_tape_n
    and out_str_n (1 int64 each), out_str (>= len + 2n + 4 uint8), out_err (1)."""
    n = idx.numel() if n is None else int(n)
    ln = buf.numel() if length is None else int(length)
    _check(lib().jsidx_tape(_ptr(buf), ln, _ptr(idx), n, _ptr(match), _ptr(out_tape), _ptr(out_tape_n),
                            _ptr(out_str), _ptr(out_str_n), _ptr(out_err), _stream(stream)))


VARIANT_NAIVE_CLASSIFY = 1
VARIANT_XOR_LOOP = 2
VARIANT_DIRECT_FLATTEN = 4
VARIANTS = {"default": 0, "naive_classify": VARIANT_NAIVE_CLASSIFY, "xor_loop": VARIANT_XOR_LOOP,
            "direct_flatten": VARIANT_DIRECT_FLATTEN}


def set_variant(variant: int) -> None:
    """jsidx_set_variant: the indexing kernel for later build calls (0 or one
    VARIANT_* flag)."""
    _check(lib().jsidx_set_variant(int(variant)))


def tile_rows(span: int) -> int:
    v = ctypes.c_uint32(0)
    _check(lib().jsidx_tile_rows(int(span), ctypes.byref(v)))
    return int(v.value)


def index(buf, stream=None):
    """Index one document held in a uint8 device tensor.

    Returns (positions int32 tensor of length n, n, flags) -- synchronises.
    """
    import torch
    dev = buf.device
    out = torch.empty(max(1, buf.numel()), dtype=torch.int32, device=dev)
    n = torch.empty(1, dtype=torch.int32, device=dev)
    err = torch.empty(1, dtype=torch.int32, device=dev)
    build(buf, out, n, err, stream)
    nn = int(n.item())
    return out[:nn], nn, int(err.item()) & 0xFFFFFFFF


def index_batch(bufs, offsets, stream=None):
    """Index a batch; returns (out_idx, out_n, out_err) device tensors."""
    import torch
    dev = bufs.device
    total = int(offsets[-1].item())
    nd = offsets.numel() - 1
    out = torch.empty(max(1, total), dtype=torch.int32, device=dev)
    n = torch.empty(nd, dtype=torch.int32, device=dev)
    err = torch.empty(nd, dtype=torch.int32, device=dev)
    build_batch(bufs, offsets, out, n, err, stream)
    return out, n, err
