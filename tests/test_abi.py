"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jsidx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jsidx_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ("jsidx_build", "jsidx_build_batch", "jsidx_reserve", "jsidx_workspace_bytes",
              "jsidx_release", "jsidx_status_string", "jsidx_stream_diag"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1902_08318_amd as jx
    lib = ctypes.CDLL(jx.library_path())
    for n in _declared():
        assert hasattr(lib, n), n
    from paper_1902_08318_amd.binding import SIGNATURES
    assert sorted(SIGNATURES) == _declared()


def test_invalid_arguments_are_rejected_without_launch():
    import paper_1902_08318_amd as jx
    lib = jx.binding.lib()
    one = ctypes.c_void_p(16)
    # NULL outputs, huge length, NULL buffer with nonzero length, ndocs == 0
    assert lib.jsidx_build(one, 10, None, one, one, None) == -1
    assert lib.jsidx_build(one, 1 << 32, one, one, one, None) == -1
    assert lib.jsidx_build(None, 5, one, one, one, None) == -1
    assert lib.jsidx_build_batch(one, one, 0, one, one, one, None) == -1
    assert lib.jsidx_build_batch(one, None, 3, one, one, one, None) == -1
    assert lib.jsidx_stream_diag(None, None) == -1
    assert lib.jsidx_status_string(-1) == b"invalid argument"
    assert lib.jsidx_workspace_bytes(0, 0) > 0
    assert lib.jsidx_workspace_bytes(1 << 30, 1) > lib.jsidx_workspace_bytes(1 << 20, 1)
    # the size depends on the bytes only (documents are found from the offsets in place)
    assert lib.jsidx_workspace_bytes(1 << 24, 1) == lib.jsidx_workspace_bytes(1 << 24, 100000)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1902_08318_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(binding.JsidxError):
        binding.lib()


def test_tile_rows_table_is_validated_on_the_host():
    """jsidx_set_tile_rows takes 0 (built-in) or 2/4/8/16 per size class and
    rejects anything else without changing the table (no device needed)."""
    import paper_1902_08318_amd as jx
    lib = jx.binding.lib()
    good = (ctypes.c_uint8 * 64)(*([0] * 10 + [2, 4, 8, 16] + [0] * 50))
    assert lib.jsidx_set_tile_rows(good, 64) == 0
    for bad in (1, 3, 5, 32, 255):
        t = (ctypes.c_uint8 * 1)(bad)
        assert lib.jsidx_set_tile_rows(t, 1) == -1
    assert lib.jsidx_set_tile_rows(good, 65) == -1
    assert lib.jsidx_set_tile_rows(None, 3) == -1
    assert lib.jsidx_set_tile_rows(None, 0) == 0
    with pytest.raises(jx.JsidxError):
        jx.set_tile_rows([3])
    jx.set_tile_rows([])
