"""jsidx_build_noalloc (the entry point for callers that cannot allocate)
against jsidx_build and the oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _both(doc: bytes, stream):
    """(positions, n, err) from jsidx_build and from jsidx_build_noalloc on
    the same device copy of doc, on one stream."""
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import binding
    dev = torch.device("cuda:0")
    buf = torch.frombuffer(bytearray(doc), dtype=torch.uint8).to(dev) if doc else torch.zeros(1, dtype=torch.uint8,
                                                                                              device=dev)
    res = []
    for fn in (jx.build, binding.build_noalloc):
        out = torch.full((max(1, len(doc)),), -1, dtype=torch.int32, device=dev)
        n = torch.full((1,), -1, dtype=torch.int32, device=dev)
        err = torch.full((1,), -1, dtype=torch.int32, device=dev)
        fn(buf, out, n, err, stream, length=len(doc))
        stream.synchronize()
        k = int(n.item())
        res.append((out[:max(0, k)].cpu().numpy().view(np.uint32).copy(), k, int(err.item()) & 0xFFFFFFFF))
    return res


def test_noalloc_equals_build_on_two_calls_the_second_smaller():
    """Two calls in a row on one stream, the second on a smaller document
    (the static workspace keeps the first call's contents): each equals
    jsidx_build and the oracle, positions, count and flags."""
    import torch
    from paper_1902_08318_amd import synth
    s = torch.cuda.Stream()
    first = synth.gen_c1(1).data  # full size, 256 MiB - 10,640 bytes
    second = synth.gen_c0(2, 300_000).data + b' "open'
    for label, doc in (("C1 full size", first), ("C0 300 KB, unclosed string", second)):
        _say(f"case: no-alloc {label}, {len(doc)} bytes")
        (bi, bn, be), (ni, nn, ne) = _both(doc, s)
        oi, oe = oracle.index(doc)
        assert bn == nn == len(oi) and be == ne == oe, (label, bn, nn, len(oi), be, ne, oe)
        assert np.array_equal(ni, bi) and np.array_equal(ni, oi), label


def test_noalloc_small_and_empty_documents():
    import torch
    s = torch.cuda.Stream()
    for doc in (b"", b"1", b'{"a":[1,2]}', b'"\\', b"[" * 70000):
        _say(f"case: no-alloc small {len(doc)} bytes")
        (bi, bn, be), (ni, nn, ne) = _both(doc, s)
        assert (bn, be) == (nn, ne) and np.array_equal(bi, ni)


def test_noalloc_rejects_documents_above_its_limit():
    """Larger than JSIDX_NOALLOC_MAX_LEN: JSIDX_E_TOO_LARGE, nothing launched."""
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import binding
    _say("case: no-alloc above the limit")
    assert binding.NOALLOC_MAX_LEN == 268435440
    buf = torch.zeros(16, dtype=torch.uint8, device="cuda:0")
    out = torch.zeros(16, dtype=torch.int32, device="cuda:0")
    n = torch.full((1,), 7, dtype=torch.int32, device="cuda:0")
    err = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(jx.JsidxError, match="too large"):
        binding.build_noalloc(buf, out, n, err, length=binding.NOALLOC_MAX_LEN + 1)
    torch.cuda.synchronize()
    assert int(n.item()) == 7  # nothing ran
