"""GPU parity of the minify pass (jsidx_minify / jsidx_minify_batch, through
the C ABI) against the oracle: kept bytes, counts and flags, bit-exact."""
import json
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_minify(data: bytes, misalign: int = 0):
    import torch
    import paper_1902_08318_amd as jx
    dev = torch.device("cuda:0")
    n = len(data)
    backing = torch.zeros(n + misalign + 64, dtype=torch.uint8, device=dev)
    if n:
        backing[misalign:misalign + n] = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    buf = backing[misalign:misalign + n]
    out = torch.full((max(1, n),), 0xEE, dtype=torch.uint8, device=dev)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=dev)
    err = torch.full((1,), -1, dtype=torch.int32, device=dev)
    jx.minify(buf, out, cnt, err, length=n)
    torch.cuda.synchronize()
    k = int(cnt.item())
    return out[:max(0, k)].cpu().numpy().tobytes(), k, int(err.item()) & 0xFFFFFFFF


def assert_minify_matches(data: bytes, misalign: int = 0, label: str = ""):
    got, n, err = gpu_minify(data, misalign)
    want, we = oracle.minify(data)
    assert n == len(want), f"{label}: kept {n} != oracle {len(want)}"
    assert err == we, f"{label}: flags {err:#x} != {we:#x}"
    if got != want:
        i = next(i for i in range(n) if got[i] != want[i])
        raise AssertionError(f"{label}: first difference at byte {i}")


def gpu_minify_batch(data: bytes, offsets: np.ndarray, lead: int = 0):
    import torch
    import paper_1902_08318_amd as jx
    dev = torch.device("cuda:0")
    arr = np.frombuffer(data, dtype=np.uint8)
    bufs = torch.zeros(arr.size + lead + 64, dtype=torch.uint8, device=dev)
    if arr.size:
        bufs[lead:lead + arr.size] = torch.from_numpy(arr.copy()).to(dev)
    offs = torch.from_numpy(offsets.astype(np.int64) + lead).to(dev)
    total = int(offsets[-1]) + lead
    out = torch.full((max(1, total),), 0xEE, dtype=torch.uint8, device=dev)
    nd = offsets.size - 1
    n = torch.full((nd,), -1, dtype=torch.int32, device=dev)
    err = torch.full((nd,), -1, dtype=torch.int32, device=dev)
    jx.minify_batch(bufs, offs, out, n, err)
    torch.cuda.synchronize()
    return out.cpu().numpy()[lead:], n.cpu().numpy().view(np.uint32), err.cpu().numpy().view(np.uint32)


def assert_minify_batch_matches(data: bytes, offsets: np.ndarray, lead: int = 0, label: str = ""):
    go, gn, ge = gpu_minify_batch(data, offsets, lead)
    oo, on, oe = oracle.minify_batch(np.frombuffer(data, dtype=np.uint8), offsets)
    assert np.array_equal(gn, on), f"{label}: counts differ"
    assert np.array_equal(ge, oe), f"{label}: flags differ"
    for d in range(offsets.size - 1):
        a = int(offsets[d])
        if not np.array_equal(go[a:a + on[d]], oo[a:a + on[d]]):
            raise AssertionError(f"{label}: document {d} differs")


def _soup(rng, n, alpha=b'"\\[]{},: \tax1\xc3\xa9\n\r'):
    a = np.frombuffer(alpha, dtype=np.uint8)
    return a[rng.integers(0, a.size, n)].tobytes()


def test_minify_small_and_json_documents():
    _say("case: minify small documents")
    for d in (b"", b" ", b"1", b' { "a b" : [ 1 , "x\\" y" ] } ', b'"\t"', b"\\ ", b'"unclosed  '):
        for mis in (0, 5):
            assert_minify_matches(d, mis, repr(d))
    obj = {"k": [1, 2.5, "a b", {"x": None, "y": "q\"r"}], "z": "é \U0001F600"}
    text = json.dumps(obj, indent=3, ensure_ascii=False).encode()
    got, n, err = gpu_minify(text)
    assert got == json.dumps(obj, separators=(",", ":"), ensure_ascii=False).encode() and err == 0


def test_minify_random_documents_across_tiles():
    rng = np.random.default_rng(77)
    for k in range(12):
        n = int(rng.integers(0, 300000))
        _say(f"case: minify soup {k} len {n}")
        assert_minify_matches(_soup(rng, n), k % 16, f"soup {k}")
    for run in (1, 2, 4095, 4097, 32769):
        d = b'[ "' + b"a " * 20000 + b"\\" * run + b'" , 7 ]  "tail"'
        assert_minify_matches(d, 3, f"backslash run {run}")


@pytest.mark.parametrize("rows", [2, 16])
def test_minify_generated_documents(rows):
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    jx.set_tile_rows([rows] * 64)
    try:
        for seed in range(3):
            doc = synth.gen_c0(seed, 1 << 20).data
            _say(f"case: minify C0 seed {seed} rows {rows}")
            assert_minify_matches(doc, seed, f"C0 {seed}")
        doc = synth.gen_c2(2, 8 << 20, pool=16).data
        assert_minify_matches(doc, 1, "C2-like 8 MiB")
    finally:
        jx.set_tile_rows([])


def test_minify_full_size_pretty_document():
    from paper_1902_08318_amd import synth
    doc = synth.gen_c2(2).data
    _say(f"case: minify C2 full size {len(doc)}")
    assert_minify_matches(doc, 0, "C2")


def test_minify_batches():
    from paper_1902_08318_amd import synth
    rng = np.random.default_rng(5)
    docs = [b"", b"  ", b' [ 1 ] ', b'"a  b', b"\\"] + [_soup(rng, int(rng.integers(0, 40000))) for _ in range(150)]
    data = b"".join(docs)
    offs = np.concatenate([[0], np.cumsum([len(x) for x in docs])]).astype(np.uint64)
    _say("case: minify mixed batch")
    assert_minify_batch_matches(data, offs, 7, "mixed")
    data, offs, _ = synth.gen_c3(3)
    _say("case: minify C3 full batch")
    assert_minify_batch_matches(data, offs, 0, "C3")
    import paper_1902_08318_amd as jx
    assert jx.diag() == 0
