"""jsidx: stage-1 JSON structural indexing on MI355X (gfx950).

Stage 1 of Langdale & Lemire, "Parsing Gigabytes of JSON per Second"
(Sec. 3.1): UTF-8 validation, escape and string-range resolution,
structural / pseudo-structural classification and flattening into uint32
positions, all in hand-written HIP kernels behind the C ABI of
include/jsidx.h.  This package only marshals arguments to that library.
"""
from .binding import (  # noqa: F401
    ERR_CAPACITY, ERR_EMPTY, ERR_OFFSETS, ERR_LITERAL, ERR_MISMATCHED, ERR_NUMBER, ERR_STRING, ERR_SYNTAX, ERR_TRAILING_ESCAPE,
    ERR_UNBALANCED, ERR_UNCLOSED_STRING, ERR_UTF8,
    JsidxError, build, build_batch, diag, index, index_batch, library_path, minify, minify_batch, release, reserve,
    VARIANTS, scopes, scopes_batch, scopes_reserve, set_tile_rows, set_variant, tape, tape_batch, tape_reserve, tile_rows, workspace_bytes,
)
