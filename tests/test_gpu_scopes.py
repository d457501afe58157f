"""GPU scope links (jsidx_scopes on the index jsidx_build wrote) against the
oracle's bracket stack and structure check, bit-exact: every link and the
flags."""
import itertools
import json
import random
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_scopes(data: bytes):
    import torch
    import paper_1902_08318_amd as jx
    dev = torch.device("cuda:0")
    n = len(data)
    buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev) if n else torch.zeros(1, dtype=torch.uint8,
                                                                                                device=dev)
    idx = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    err = torch.empty(1, dtype=torch.int32, device=dev)
    jx.build(buf, idx, cnt, err, length=n)
    k = int(cnt.item())
    match = torch.full((max(1, k),), 0x5A5A5A5A, dtype=torch.int32, device=dev)
    serr = torch.full((1,), -1, dtype=torch.int32, device=dev)
    jx.scopes(buf, idx, match, serr, n=k, length=n)
    torch.cuda.synchronize()
    return (idx[:k].cpu().numpy().view(np.uint32), match[:k].cpu().numpy().view(np.uint32),
            int(serr.item()) & 0xFFFFFFFF)


def assert_scopes_match(data: bytes, label: str):
    idx, m, e = gpu_scopes(data)
    oi, _ = oracle.index(data)
    assert np.array_equal(idx, oi), f"{label}: index differs"
    om, oe = oracle.scopes(data, oi)
    oe |= oracle.structure(data, oi)
    assert e == oe, f"{label}: flags {e:#x} != {oe:#x}"
    bad = np.nonzero(m != om)[0]
    assert bad.size == 0, f"{label}: {bad.size} links differ, first entry {bad[0] if bad.size else -1}"


def test_scopes_small_and_invalid():
    _say("case: scopes small")
    for d in (b"", b"7", b"[]", b'{"a":[1,{"b":[]}]}', b"[}", b"]", b"[[", b"[ ] ]", b"{ [ } ]", b'"[" ]'):
        assert_scopes_match(d, repr(d))


def test_scopes_generated_documents():
    from paper_1902_08318_amd import synth
    for name, doc in (("C0", synth.gen_c0(0, 1 << 20).data), ("C1 8 MiB", synth.gen_c1(1, 8 << 20, pool=256).data),
                      ("C2 8 MiB", synth.gen_c2(2, 8 << 20, pool=16).data)):
        _say(f"case: scopes {name}")
        assert_scopes_match(doc, name)
        assert_scopes_match(doc[:-1], name + " cut")
        assert_scopes_match(doc.replace(b"}", b"]", 3), name + " mismatched")


def test_scopes_deep_and_wide():
    _say("case: scopes deep and wide")
    assert_scopes_match(b"[" * 100000 + b"1" + b"]" * 100000, "depth 100000")
    assert_scopes_match(b"[" * 70000 + b"]" * 50000, "unbalanced deep")
    rng = random.Random(9)

    def val(d):
        r = rng.random()
        if d > 9 or r < 0.4:
            return rng.choice([1, "x]", None, "{"])
        if r < 0.7:
            return [val(d + 1) for _ in range(rng.randrange(0, 7))]
        return {f"k{i}": val(d + 1) for i in range(rng.randrange(0, 7))}

    doc = json.dumps([val(0) for _ in range(20000)], indent=1).encode()
    assert_scopes_match(doc, "random nested")


def test_scopes_full_size_c1():
    from paper_1902_08318_amd import synth
    doc = synth.gen_c1(1).data
    _say(f"case: scopes C1 full size {len(doc)}")
    assert_scopes_match(doc, "C1")


def test_structure_of_every_short_token_sequence():
    """Every sequence of up to 4 tokens, and 3000 random ones of 5 to 9."""
    _say("case: structure of token sequences up to 4")
    toks = ["{", "}", "[", "]", ":", ",", '"s"', "1"]
    for n in range(0, 5):
        for seq in itertools.product(toks, repeat=n):
            d = " ".join(seq).encode()
            assert_scopes_match(d, repr(d))
    _say("case: structure of random token sequences of 5 to 9")
    rng = random.Random(31)
    for _ in range(3000):
        d = " ".join(rng.choice(toks) for _ in range(rng.randrange(5, 10))).encode()
        assert_scopes_match(d, repr(d))


def test_structure_edits_of_generated_documents():
    from paper_1902_08318_amd import synth
    rng = random.Random(4)
    for name, doc in (("C0", synth.gen_c0(3, 1 << 20).data), ("C2 4 MiB", synth.gen_c2(2, 4 << 20, pool=16).data)):
        text = doc.decode("utf-8")
        oi, _ = oracle.index(doc)
        assert oracle.structure(doc, oi) == 0
        for k in range(12):
            p = int(oi[rng.randrange(oi.size)])
            ch = rng.choice(["{", "}", "[", "]", ":", ",", " ", '"x"', "1"])
            edited = (doc[:p] + ch.encode() + doc[p + 1:]) if k % 2 else (doc[:p] + b" " + ch.encode() + b" " + doc[p:])
            _say(f"case: structure edit {name} {k} at {p}")
            assert_scopes_match(edited, f"{name} edit {k}")
