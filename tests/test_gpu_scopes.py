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


def _oracle_batch_scopes(data: bytes, offs: np.ndarray, oi: np.ndarray, on: np.ndarray):
    """Per-document oracle links (batch layout) and flags."""
    em = np.full(max(1, int(offs[-1])), 0xFFFFFFFF, dtype=np.uint32)
    ee = np.zeros(offs.size - 1, dtype=np.uint32)
    for d in range(offs.size - 1):
        a, b = int(offs[d]), int(offs[d + 1])
        ix = oi[a:a + on[d]]
        m, e = oracle.scopes(data[a:b], ix)
        ee[d] = e | oracle.structure(data[a:b], ix)
        em[a:a + on[d]] = m
    return em, ee


def gpu_scopes_batch(data: bytes, offs: np.ndarray, reserve_entries=None, stream=None):
    """jsidx_build_batch, then jsidx_scopes_batch over its index (after
    jsidx_scopes_reserve for the batch's entries, or reserve_entries)."""
    import torch
    import paper_1902_08318_amd as jx
    dev = torch.device("cuda:0")
    total = int(offs[-1])
    nd = offs.size - 1
    buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    o = torch.from_numpy(offs.astype(np.int64)).to(dev)
    idx = torch.empty(max(1, total), dtype=torch.int32, device=dev)
    cnt = torch.empty(nd, dtype=torch.int32, device=dev)
    err = torch.empty(nd, dtype=torch.int32, device=dev)
    jx.build_batch(buf, o, idx, cnt, err, stream)
    torch.cuda.synchronize()
    on = cnt.cpu().numpy().view(np.uint32).copy()
    jx.scopes_reserve(int(on.sum()) if reserve_entries is None else reserve_entries, nd, stream)
    match = torch.full((max(1, total),), 0x5A5A5A5A, dtype=torch.int32, device=dev)
    serr = torch.full((nd,), -1, dtype=torch.int32, device=dev)
    jx.scopes_batch(buf, o, idx, cnt, match, serr, stream)
    torch.cuda.synchronize()
    return (idx.cpu().numpy().view(np.uint32), on, match.cpu().numpy().view(np.uint32),
            serr.cpu().numpy().view(np.uint32))


def _check_batch(data: bytes, offs: np.ndarray, label: str):
    gi, gn, gm, ge = gpu_scopes_batch(data, offs)
    oi, on, _ = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert np.array_equal(gn, on), f"{label}: counts differ"
    em, ee = _oracle_batch_scopes(data, offs, oi, on)
    bad = np.nonzero(ge != ee)[0]
    assert bad.size == 0, f"{label}: flags of {bad.size} documents differ, first {bad[0]}: {ge[bad[0]]:#x} != {ee[bad[0]]:#x}"
    for d in range(offs.size - 1):
        a = int(offs[d])
        if not np.array_equal(gm[a:a + on[d]], em[a:a + on[d]]):
            raise AssertionError(f"{label}: links of document {d} differ")


def test_scopes_batch_mixed_documents():
    """Small valid and invalid documents, empty ones, unclosed openers whose
    search must stop at their own document, and documents of more than one
    chunk (4096 entries), in one batched call."""
    rng = random.Random(5)
    small = [b"", b"1", b"[]", b"{}", b"[}", b"]", b"[[", b"[ ] ]", b'{"a":[1,{"b":[]}]}', b"{ [ } ]",
             b"]]]][[[[", b"[" * 50 + b"]" * 49, b'{"a":1,"b":[2,3]}', b"[1,2", b'{"k" 1}', b",", b'"s"', b"  "]

    def val(dp):
        r = rng.random()
        if dp > 6 or r < 0.4:
            return rng.choice([1, "s]", None, True])
        if r < 0.7:
            return [val(dp + 1) for _ in range(rng.randrange(0, 5))]
        return {f"k{i}": val(dp + 1) for i in range(rng.randrange(0, 5))}

    docs = []
    for k in range(3000):
        if k % 3 == 0:
            docs.append(rng.choice(small))
        else:
            d = json.dumps(val(0), separators=(",", ":")).encode()
            docs.append(d[:-1] if k % 7 == 0 and len(d) > 2 else d)
    big = json.dumps([val(0) for _ in range(3000)], separators=(",", ":")).encode()
    for pos in (100, 1500, 2999):
        docs.insert(pos, big)
    docs.insert(700, big[:-1])
    docs.insert(701, b"[" * 6000 + b"]" * 5000)
    data = b"".join(docs)
    offs = np.zeros(len(docs) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in docs], out=offs[1:])
    _say(f"case: scopes batch mixed, {len(docs)} documents, {len(data)} bytes")
    _check_batch(data, offs, "mixed")


def test_scopes_batch_full_c3():
    """The whole C3 batch (100,000 documents, 1% corrupted): every document's
    links and flags equal the oracle's for that document alone."""
    from paper_1902_08318_amd import synth
    data, offs, _ = synth.gen_c3(3)
    _say(f"case: scopes batch C3, {offs.size - 1} documents, {len(data)} bytes")
    _check_batch(data, offs, "C3")


def test_scopes_batch_capacity_flag():
    import torch
    docs = [b"[1,2]", b'{"a":[]}', b"[[[]]]"]
    data = b"".join(docs)
    offs = np.array([0, 5, 13, 19], dtype=np.uint64)
    _say("case: scopes batch over its reservation")
    s = torch.cuda.Stream()
    gi, gn, gm, ge = gpu_scopes_batch(data, offs, reserve_entries=3, stream=s)
    assert int(gn.sum()) > 3 and np.all(ge == 0x80000000)


def test_scopes_batch_replayed_from_graph():
    """After jsidx_scopes_reserve the batched call is captured in a HIP graph
    and replayed on new batches (written between replays, same document
    count); every replay equals an eager call and the oracle."""
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    dev = torch.device("cuda:0")
    ndocs, cap = 600, 4 << 20
    batches = []
    for sd in (41, 42, 43):
        data, o, _ = synth.gen_c3(sd, ndocs=ndocs, pool=80, median=1024, hi=16384, corrupt_frac=0.05)
        assert int(o[-1]) <= cap
        batches.append((data, o))
    s = torch.cuda.Stream()
    bufs = torch.zeros(cap, dtype=torch.uint8, device=dev)
    offs = torch.zeros(ndocs + 1, dtype=torch.int64, device=dev)
    idx = torch.zeros(cap, dtype=torch.int32, device=dev)
    cnt = torch.zeros(ndocs, dtype=torch.int32, device=dev)
    err = torch.zeros(ndocs, dtype=torch.int32, device=dev)
    match = torch.zeros(cap, dtype=torch.int32, device=dev)
    serr = torch.zeros(ndocs, dtype=torch.int32, device=dev)

    def load(k):
        data, o = batches[k]
        bufs[:len(data)].copy_(torch.frombuffer(bytearray(data), dtype=torch.uint8))
        offs.copy_(torch.from_numpy(o.astype(np.int64)))
        jx.build_batch(bufs, offs, idx, cnt, err, s)
        match.fill_(-1)
        serr.fill_(-1)

    with torch.cuda.stream(s):
        jx.reserve(cap, s)
        jx.scopes_reserve(cap, ndocs, s)
        load(0)
        jx.scopes_batch(bufs, offs, idx, cnt, match, serr, s)  # eager warm-up on the capture stream
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        jx.scopes_batch(bufs, offs, idx, cnt, match, serr, s)
    for r in range(5):
        k = r % len(batches)
        data, o = batches[k]
        _say(f"case: scopes batch graph replay {r} (batch {k})")
        with torch.cuda.stream(s):
            load(k)
            jx.scopes_batch(bufs, offs, idx, cnt, match, serr, s)
        s.synchronize()
        e_m, e_e = match.clone(), serr.clone()
        with torch.cuda.stream(s):
            match.fill_(-1)
            serr.fill_(-1)
        s.synchronize()
        g.replay()
        s.synchronize()
        assert torch.equal(serr, e_e) and torch.equal(match[:len(data)], e_m[:len(data)]), f"replay {r}"
        on = cnt.cpu().numpy().view(np.uint32)
        oi = idx.cpu().numpy().view(np.uint32)
        em, ee = _oracle_batch_scopes(data, o, oi, on)
        assert np.array_equal(serr.cpu().numpy().view(np.uint32), ee), f"replay {r}: flags"
        gm = match.cpu().numpy().view(np.uint32)
        for d in range(ndocs):
            a = int(o[d])
            assert np.array_equal(gm[a:a + on[d]], em[a:a + on[d]]), f"replay {r}: document {d}"
